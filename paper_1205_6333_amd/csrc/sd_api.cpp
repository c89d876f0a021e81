// sd_api.cpp -- the C ABI declared in include/sd.h: argument checks, library
// workspace, launch configuration and the host side of the time loop.
#include "sd.h"
#include "sd_internal.h"
#include "sd_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace sd {

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

sd_status fail(sd_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

sd_status ok()
{
    return SD_OK;
}

sd_status check_params(const sd_params* p)
{
    if (!p) return fail(SD_EINVAL, "params is NULL");
    if (!(p->a > 0.0) || !std::isfinite(p->a)) return fail(SD_EINVAL, "a must be finite and > 0");
    if (!(p->eta > 0.0) || !std::isfinite(p->eta))
        return fail(SD_EINVAL, "eta must be finite and > 0");
    if (p->tensor != SD_RPY && p->tensor != SD_OSEEN) return fail(SD_EINVAL, "unknown tensor");
    if (p->overlap != SD_OVERLAP_NONE && p->overlap != SD_OVERLAP_RPY)
        return fail(SD_EINVAL, "unknown overlap mode");
    for (int k = 0; k < 3; ++k)
        if (!(p->box[k] >= 0.0) || !std::isfinite(p->box[k]))
            return fail(SD_EINVAL, "box sides must be finite and >= 0");
    if (p->box[0] != 0.0 || p->box[1] != 0.0 || p->box[2] != 0.0) {
        if (p->box[0] != p->box[1] || p->box[0] != p->box[2])
            return fail(SD_EUNSUPPORTED, "the box must be cubic (three equal sides) or absent");
        if (!(p->box[0] > 2.0 * p->a))
            return fail(SD_EINVAL, "the box side must exceed the sphere diameter 2a");
    }
    return SD_OK;
}

sd_status check_free_space(const sd_params* p, const char* what)
{
    if (box_side(p) > 0.0) return fail(SD_EUNSUPPORTED, "%s does not support a periodic box", what);
    return SD_OK;
}

sd_status check_n(int64_t n)
{
    if (n < 1) return fail(SD_EINVAL, "n must be >= 1 (got %lld)", (long long)n);
    if (n > MAX_N) return fail(SD_EINVAL, "n must be <= %lld (got %lld)", (long long)MAX_N,
                               (long long)n);
    return SD_OK;
}

sd_status check_precision(int32_t prec)
{
    if (prec != SD_FP32_KAHAN && prec != SD_FP64 && prec != SD_FP32_PLAIN)
        return fail(SD_EINVAL, "unknown precision %d", prec);
    return SD_OK;
}

sd_status check_ptr(const void* ptr, size_t align, const char* name)
{
    if (!ptr) return fail(SD_EINVAL, "%s is NULL", name);
    if ((uintptr_t)ptr % align) return fail(SD_EALIGN, "%s is not %zu-byte aligned", name, align);
    return SD_OK;
}

size_t vec4_align(int32_t prec)
{
    return prec == SD_FP64 ? 32 : 16;
}

// --------------------------------------------------------------- device info

static std::mutex g_mu;

struct DeviceInfo {
    int cus = 0;
};
static std::map<int, DeviceInfo> g_dev;

int device_cus()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(g_mu);
    auto& d = g_dev[dev];
    if (d.cus == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            d.cus = prop.multiProcessorCount;
        else
            d.cus = 256;
    }
    return d.cus;
}

// ---------------------------------------------------------------- workspace

struct Buffer {
    void* ptr = nullptr;
    size_t bytes = 0;
};

struct Workspace {
    Buffer slot[WS_COUNT];
    // buffers replaced by larger ones: work already enqueued may still use
    // them, so they are freed only by sd_release (which waits for the device)
    std::vector<void*> retired;
};
static std::map<int, Workspace> g_ws;

// Returns a device buffer of at least `bytes` for workspace slot `which` on the
// current device (grow-only, by at least 1.5x; a new buffer is zeroed).  The
// buffer it replaces stays allocated until sd_release, so growing never waits
// for the device.
sd_status ws_get(int which, size_t bytes, void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SD_EDEVICE, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace& w = g_ws[dev];
    Buffer& b = w.slot[which];
    if (b.bytes < bytes) {
        size_t want = std::max(bytes, (size_t)4096);
        if (b.bytes) want = std::max(want, b.bytes + b.bytes / 2);
        want = (want + 4095) & ~(size_t)4095;
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SD_ENOMEM, "workspace allocation of %zu bytes failed", want);
        }
        if (hipMemset(p, 0, want) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(p);
            return fail(SD_EDEVICE, "workspace initialisation failed");
        }
        if (b.ptr) w.retired.push_back(b.ptr);
        b.ptr = p;
        b.bytes = want;
    }
    *out = b.ptr;
    return SD_OK;
}

static sd_status ws_release_all()
{
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_ws) {
        if (hipSetDevice(kv.first) != hipSuccess) continue;
        (void)hipDeviceSynchronize();
        for (auto& b : kv.second.slot)
            if (b.ptr) {
                (void)hipFree(b.ptr);
                b.ptr = nullptr;
                b.bytes = 0;
            }
        for (void* r : kv.second.retired) (void)hipFree(r);
        kv.second.retired.clear();
    }
    (void)hipSetDevice(cur);
    return SD_OK;
}

// ------------------------------------------------------------ configuration

struct ConfigTable {
    bool forced = false;
    sd_kernel_config forced_cfg{};
    // tuned entries by size class (floor(log2 n))
    std::map<int, sd_kernel_config> tuned;
};
static ConfigTable g_cfg[3];

static int size_class(int64_t n)
{
    int c = 0;
    while ((int64_t(1) << (c + 1)) <= n) ++c;
    return c;
}

bool sym_fits(int64_t n, int block)
{
    if (n > INT32_MAX) return false;
    const SymShape sh = sym_shape((int)n, block, 1, 1);
    return sym_jpart_floats(sh) * sizeof(float) <= SYM_WORKSPACE_CAP;
}

sd_kernel_config default_config(int32_t prec, int64_t n)
{
    sd_kernel_config c;
    c.variant = 0;
    // Below n = 4096, 256-lane groups (an i-block and a j-tile per work-group)
    // cannot fill the chip: 64-lane groups give 16x as many.  (Measured on the
    // fcc start: n = 256 0.024 -> 0.014 ms per step, n = 2048 0.027 -> 0.024;
    // at n = 5324 128-lane groups were slower than 256.)  The Kahan block of 8
    // needs groups of at least 128 lanes.
    c.block = n >= 4096 ? 256 : 64;
    c.ilp = 1;
    c.kahan_block = (prec == SD_FP32_PLAIN) ? 0 : (c.block >= 128 ? 8 : 4);
    if (prec == SD_FP64) {
        c.variant = 0;
        c.kahan_block = 0;
    }
    // about 32 waves per SIMD over the launch (several rounds of resident
    // waves, so the last round's imbalance is a small fraction of the run)
    const int cus = device_cus();
    const int64_t iblocks = (n + c.block * c.ilp - 1) / (c.block * c.ilp);
    const int64_t target = (int64_t)cus * 4 * 32 / (c.block / 64);
    int64_t s = std::max<int64_t>(1, (target + iblocks - 1) / iblocks);
    const int64_t tiles = (n + c.block - 1) / c.block;
    s = std::min<int64_t>(s, tiles);
    s = std::min<int64_t>(s, 512);
    c.splits = (int32_t)s;
    // From n = SYM_MIN_N on, the pair-symmetric kernel (each pair of particles
    // in different blocks evaluated once) with two particles per lane,
    // whenever its j-side workspace fits.  Measured (ms per pair-kernel
    // launch, one box): N = 65536: variant 0 2.10, variant 2 1.45;
    // N = 32768: 0.551 vs 0.388; N = 24576: 0.332 vs 0.229; N = 16384: 0.166
    // vs 0.116.
    if (prec != SD_FP64 && n >= SYM_MIN_N && sym_fits(n, 2 * c.block)) {
        c.variant = 2;
        c.ilp = 2;
        // (N = 16384: 0.119 ms per launch at 16 splits, 0.116 at 32, 0.120 at 64)
        c.splits = std::min<int32_t>(c.splits, 32);
        // Kahan blocks of 32 terms select the chunk loop in generated assembly
        // (N = 65536: 1.45 ms per pair-kernel launch against 1.73 for the
        // compiled loop with blocks of 8)
        if (prec == SD_FP32_KAHAN && c.block == 256) c.kahan_block = 32;
    }
    return c;
}

sd_kernel_config choose_config(int32_t prec, int64_t n)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        const ConfigTable& t = g_cfg[prec];
        sd_kernel_config c{};
        bool have = false;
        if (t.forced) {
            c = t.forced_cfg;
            have = true;
        } else {
            auto it = t.tuned.find(size_class(n));
            if (it != t.tuned.end()) {
                c = it->second;
                // keep the split count proportional to the size class
                const int64_t tiles = (n + c.block - 1) / c.block;
                if (c.splits > tiles) c.splits = (int32_t)tiles;
                have = true;
            }
        }
        // a forced or tuned variant-2 shape whose j-side workspace for this n
        // exceeds the cap falls back to the automatic configuration
        if (have && !(c.variant == 2 && !sym_fits(n, c.block * c.ilp))) return c;
    }
    return default_config(prec, n);
}

void set_tuned_config(int32_t prec, int64_t n, const sd_kernel_config& c)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_cfg[prec].tuned[size_class(n)] = c;
}

sd_status check_config(int32_t prec, const sd_kernel_config& c)
{
    if (c.block != 64 && c.block != 128 && c.block != 256 && !(c.variant == 2 && c.block == 512))
        return fail(SD_EINVAL, "block must be 64, 128 or 256 (or 512 with variant 2)");
    if (c.kahan_block == 8 && c.block < 128)
        return fail(SD_EINVAL, "kahan_block 8 needs block >= 128");
    if (c.splits < 1) return fail(SD_EINVAL, "splits must be >= 1");
    if (c.variant < 0 || c.variant > 2) return fail(SD_EINVAL, "variant must be 0, 1 or 2");
    if (c.ilp != 1 && c.ilp != 2) return fail(SD_EINVAL, "ilp must be 1 or 2");
    if (c.variant == 2) {
        if (prec == SD_FP64) return fail(SD_EINVAL, "variant 2 is an FP32 kernel");
        if (c.block != 128 && c.block != 256 && c.block != 512)
            return fail(SD_EINVAL, "variant 2 needs block 128, 256 or 512");
        if (c.block * c.ilp > 512) return fail(SD_EINVAL, "variant 2 needs block * ilp <= 512");
        if (c.kahan_block != 0 && c.kahan_block != 4 && c.kahan_block != 8 &&
            c.kahan_block != 16 && c.kahan_block != 32)
            return fail(SD_EINVAL, "variant 2 needs kahan_block 0, 4, 8, 16 or 32");
        if ((c.kahan_block == 16 || c.kahan_block == 32) && !(c.block == 256 && c.ilp == 2))
            return fail(SD_EINVAL, "kahan_block 16 or 32 needs block 256 and ilp 2");
    }
    if (prec == SD_FP64) {
        if (c.variant != 0 || c.ilp != 1)
            return fail(SD_EINVAL, "the FP64 path has variant 0 and ilp 1 only");
    } else if (prec == SD_FP32_PLAIN) {
        if (c.kahan_block != 0) return fail(SD_EINVAL, "kahan_block must be 0 for SD_FP32_PLAIN");
    } else if (c.kahan_block != 1 && c.kahan_block != 2 && c.kahan_block != 4 &&
               c.kahan_block != 8 &&
               !(c.variant == 2 && (c.kahan_block == 16 || c.kahan_block == 32))) {
        return fail(SD_EINVAL, "kahan_block must be 1, 2, 4 or 8 (16 or 32 with variant 2) for "
                               "SD_FP32_KAHAN");
    }
    return SD_OK;
}

// ---------------------------------------------------------------- profiling

struct Profile {
    std::atomic<bool> on{ false };   // read without the lock on every launch
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    int64_t launches = 0;
    double total_ms = 0.0;
    std::vector<float> times;        // per launch, the first PROF_KEEP since the reset
};
constexpr size_t PROF_KEEP = 1 << 16;
static Profile g_prof;

static void prof_begin(hipStream_t st, hipEvent_t* a)
{
    *a = nullptr;
    if (!g_prof.on) return;
    if (hipEventCreate(a) != hipSuccess) {
        *a = nullptr;
        return;
    }
    (void)hipEventRecord(*a, st);
}

static void prof_end(hipStream_t st, hipEvent_t a)
{
    if (!a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof.pending.emplace_back(a, b);
}

// ----------------------------------------------------------- product launch

PairConst pair_const(const sd_params* p)
{
    return make_pair_const(p->a, p->eta, p->tensor, p->overlap, box_side(p));
}

// Launch the pair kernel for n particles; returns the number of splits used
// through *splits_out.  partial is sized by the caller via partial_bytes().
sd_status run_pair(const sd_params* p, int64_t n, const void* pos, const void* frc,
                   const double* x64, int32_t prec, double* partial, const PairLaunch& L,
                   hipStream_t st, double* vel, bool* merged)
{
    if (merged) *merged = false;
    const PairConst pc = pair_const(p);
    hipEvent_t ev;
    prof_begin(st, &ev);
    hipError_t e;
    if (prec == SD_FP64)
        e = launch_pair_f64(L, p->tensor, (const double4*)pos, (const double4*)frc, (int)n, pc,
                            partial, st);
    else
        e = launch_pair_f32(L, p->tensor, L.acc, (const float4*)pos, (const float4*)frc, x64,
                            (int)n, pc, partial, st);
    prof_end(st, ev);
    const bool fuse = vel && prec != SD_FP64 && L.variant == 2;
    if (e == hipSuccess && prec != SD_FP64)
        e = launch_pair_fold(L, p->tensor, (const float4*)pos, (const float4*)frc, x64, (int)n, pc,
                             partial, st, 1.0 / (6.0 * M_PI * p->eta * p->a),
                             fuse ? vel : nullptr);
    if (e == hipSuccess && fuse && merged) *merged = true;
    if (e != hipSuccess) return fail(SD_EDEVICE, "pair kernel launch: %s", hipGetErrorString(e));
    return SD_OK;
}

PairLaunch plan_pair(int32_t prec, int64_t n)
{
    const sd_kernel_config c = choose_config(prec, n);
    PairLaunch L = shape_pair_launch((int)n, c.variant, c.block, c.splits, c.ilp, device_cus());
    L.acc = (prec == SD_FP64) ? 0 : c.kahan_block;
    if (prec == SD_FP32_PLAIN) L.acc = 0;
    return L;
}

size_t partial_bytes(const PairLaunch& L, int64_t n)
{
    if (L.variant == 2) return sym_workspace_bytes(L, n);
    return (size_t)L.splits * 3 * (size_t)n * sizeof(double);
}

}  // namespace sd

// ------------------------------------------------------- graph-captured loop
//
// The time loop of sd_run is launch-bound for small n (two short kernels per
// step).  Chunks of RUN_CHUNK steps [stage, (pair kernel, merge + integrate
// + staging) x RUN_CHUNK] are captured once into a HIP graph on a private
// capture stream and replayed on the caller's stream; a chunk holds only
// kernel nodes.  The graph is cached per device and rebuilt when anything it
// captured changes (pointers, sizes, parameters, launch shape, workspace).
namespace {

constexpr int RUN_CHUNK = 16;

struct RunKey {
    sd_params p{};
    int64_t n = 0;
    double* x = nullptr;
    const void* force = nullptr;
    double* v_prev = nullptr;
    double dt = 0.0;
    int32_t integ = -1, mode = -1, prec = -1;
    sd::PairLaunch L{};
    void* partial = nullptr;
    void* stage = nullptr;
    bool operator==(const RunKey& o) const { return std::memcmp(this, &o, sizeof(RunKey)) == 0; }
};

struct RunGraph {
    RunKey key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    hipEvent_t done = nullptr;  // recorded after the last replay
};

std::mutex g_rg_mu;
std::map<int, RunGraph> g_rg;
std::atomic<int32_t> g_graph_mode{ 1 };   // 0 off, 1 automatic (n <= RUN_GRAPH_AUTO_N), 2 always
constexpr int64_t RUN_GRAPH_AUTO_N = 16384;

// Waits for the last replay before the executable graph is destroyed (a
// rebuild may come from a call on another stream).
void drop_run_graph(RunGraph& g)
{
    if (g.exec && g.done) (void)hipEventSynchronize(g.done);
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
    g.key = RunKey();
}

}  // namespace

namespace sd {
void run_graphs_release()
{
    std::lock_guard<std::mutex> lk(g_rg_mu);
    for (auto& kv : g_rg) {
        drop_run_graph(kv.second);
        if (kv.second.cap) (void)hipStreamDestroy(kv.second.cap);
        if (kv.second.done) (void)hipEventDestroy(kv.second.done);
        kv.second.cap = nullptr;
        kv.second.done = nullptr;
    }
}
}  // namespace sd

using namespace sd;

// ====================================================================== ABI

extern "C" {

sd_status mobility_apply(const sd_params* p, int64_t n, const void* pos, const void* force,
                         double* vel, int32_t precision, void* stream)
{
    sd_status st;
    if ((st = check_params(p)) || (st = check_n(n)) || (st = check_precision(precision))) return st;
    const size_t al = vec4_align(precision);
    if ((st = check_ptr(pos, al, "pos")) || (st = check_ptr(force, al, "force")) ||
        (st = check_ptr(vel, 8, "vel")))
        return st;
    hipStream_t hs = (hipStream_t)stream;
    const PairLaunch L = plan_pair(precision, n);
    void* partial = nullptr;
    if ((st = ws_get(WS_PARTIAL, partial_bytes(L, n), &partial))) return st;
    const void* pos_k = pos;
    if (box_side(p) > 0.0 && precision != SD_FP64) {  // fixed-point records for the box
        void* q = nullptr;
        if ((st = ws_get(WS_QPOS, (size_t)n * 16, &q))) return st;
        hipError_t e = launch_stage_q_from_f32((const float4*)pos, (float4*)q, (int)n,
                                               box_side(p), hs);
        if (e != hipSuccess) return fail(SD_EDEVICE, "stage launch: %s", hipGetErrorString(e));
        pos_k = q;
    }
    bool merged = false;
    if ((st = run_pair(p, n, pos_k, force, nullptr, precision, (double*)partial, L, hs, vel,
                       &merged)))
        return st;
    if (merged) return SD_OK;   // the pair-symmetric kernel's fold wrote vel
    hipError_t e = (precision == SD_FP64)
                       ? launch_merge_f64((double*)partial, L.splits, (int)n, (const double4*)force,
                                          1.0 / (6.0 * M_PI * p->eta * p->a), vel, hs)
                       : launch_merge_f32((double*)partial, L.splits, (int)n, (const float4*)force,
                                          1.0 / (6.0 * M_PI * p->eta * p->a), vel, hs);
    if (e != hipSuccess) return fail(SD_EDEVICE, "merge kernel launch: %s", hipGetErrorString(e));
    return SD_OK;
}

// One time step from x (FP64).  pos_stage holds the staged copy of x on entry
// when `staged` is true.
static sd_status step_impl(const sd_params* p, int64_t n, double* x, const void* force,
                           double* v_prev, double* v_out, double dt, int64_t step_index,
                           int32_t integrator, int32_t prec, void* pos_stage, bool staged,
                           bool stage_next, double* partial, const PairLaunch& L, hipStream_t hs)
{
    sd_status st;
    hipError_t e;
    if (!staged) {
        e = (prec == SD_FP64) ? launch_stage_f64(x, (double4*)pos_stage, (int)n, hs)
                              : launch_stage_f32(x, (float4*)pos_stage, (int)n, box_side(p), hs);
        if (e != hipSuccess) return fail(SD_EDEVICE, "stage launch: %s", hipGetErrorString(e));
    }
    if ((st = run_pair(p, n, pos_stage, force, prec == SD_FP64 ? nullptr : x, prec, partial, L,
                       hs)))
        return st;
    const int mode = (integrator == SD_EULER) ? 0 : (step_index == 0 ? 1 : 2);
    const double mu0 = 1.0 / (6.0 * M_PI * p->eta * p->a);
    if (prec == SD_FP64)
        e = launch_merge_integrate_f64(partial, L.splits, (int)n, (const double4*)force, mu0, x,
                                       v_prev, v_out, dt, mode,
                                       stage_next ? (double4*)pos_stage : nullptr, hs);
    else
        e = launch_merge_integrate_f32(partial, L.splits, (int)n, (const float4*)force, mu0, x,
                                       v_prev, v_out, dt, mode,
                                       stage_next ? (float4*)pos_stage : nullptr, box_side(p), hs);
    if (e != hipSuccess) return fail(SD_EDEVICE, "integrate launch: %s", hipGetErrorString(e));
    return SD_OK;
}

static sd_status check_step_args(const sd_params* p, int64_t n, const double* x, const void* force,
                                 const double* v_prev, double dt, int32_t integrator,
                                 int32_t precision)
{
    sd_status st;
    if ((st = check_params(p)) || (st = check_n(n)) || (st = check_precision(precision))) return st;
    if ((st = check_ptr(x, 8, "x")) || (st = check_ptr(force, vec4_align(precision), "force")))
        return st;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SD_EINVAL, "dt must be finite and > 0");
    if (integrator != SD_EULER && integrator != SD_AB2) return fail(SD_EINVAL, "unknown integrator");
    if (integrator == SD_AB2 && (st = check_ptr(v_prev, 8, "v_prev"))) return st;
    if (v_prev && (uintptr_t)v_prev % 8) return fail(SD_EALIGN, "v_prev is not 8-byte aligned");
    return SD_OK;
}

sd_status sd_step(const sd_params* p, int64_t n, double* x, const void* force, double* v_prev,
                  double* v_out, double dt, int64_t step_index, int32_t integrator,
                  int32_t precision, void* stream)
{
    sd_status st;
    if ((st = check_step_args(p, n, x, force, v_prev, dt, integrator, precision))) return st;
    if (step_index < 0) return fail(SD_EINVAL, "step_index must be >= 0");
    if (v_out && (uintptr_t)v_out % 8) return fail(SD_EALIGN, "v_out is not 8-byte aligned");
    hipStream_t hs = (hipStream_t)stream;
    const PairLaunch L = plan_pair(precision, n);
    void *partial = nullptr, *stage = nullptr;
    if ((st = ws_get(WS_PARTIAL, partial_bytes(L, n), &partial)) ||
        (st = ws_get(WS_STAGE, (size_t)n * (precision == SD_FP64 ? 32 : 16), &stage)))
        return st;
    return step_impl(p, n, x, force, integrator == SD_AB2 ? v_prev : nullptr, v_out, dt,
                     step_index, integrator, precision, stage, false, false, (double*)partial, L,
                     hs);
}

sd_status sd_run(const sd_params* p, int64_t n, double* x, const void* force, double* v_prev,
                 double dt, int64_t steps, int64_t step0, int32_t integrator, int32_t precision,
                 double* x_checkpoints, int64_t checkpoint_every, void* stream)
{
    sd_status st;
    if ((st = check_step_args(p, n, x, force, v_prev, dt, integrator, precision))) return st;
    if (steps < 0 || step0 < 0) return fail(SD_EINVAL, "steps and step0 must be >= 0");
    if (x_checkpoints) {
        if ((uintptr_t)x_checkpoints % 8) return fail(SD_EALIGN, "x_checkpoints misaligned");
        if (checkpoint_every < 1) return fail(SD_EINVAL, "checkpoint_every must be >= 1");
    }
    hipStream_t hs = (hipStream_t)stream;
    const size_t frame = 3 * (size_t)n * sizeof(double);
    if (x_checkpoints && hipMemcpyAsync(x_checkpoints, x, frame, hipMemcpyDeviceToDevice, hs) !=
                             hipSuccess)
        return fail(SD_EDEVICE, "checkpoint copy failed");
    if (steps == 0) return SD_OK;
    const PairLaunch L = plan_pair(precision, n);
    void *partial = nullptr, *stage = nullptr;
    if ((st = ws_get(WS_PARTIAL, partial_bytes(L, n), &partial)) ||
        (st = ws_get(WS_STAGE, (size_t)n * (precision == SD_FP64 ? 32 : 16), &stage)))
        return st;
    double* vp = integrator == SD_AB2 ? v_prev : nullptr;
    int64_t done = 0;
    const int32_t gmode = g_graph_mode.load();
    const bool graphed = !x_checkpoints && !g_prof.on && steps >= 2 * RUN_CHUNK &&
                         (gmode == 2 || (gmode == 1 && n <= RUN_GRAPH_AUTO_N));
    if (graphed) {
        // the first AB2 step (an Euler step that stores v_prev) stays eager
        if (integrator == SD_AB2 && step0 == 0) {
            if ((st = step_impl(p, n, x, force, vp, nullptr, dt, 0, integrator, precision, stage,
                                false, false, (double*)partial, L, hs)))
                return st;
            done = 1;
        }
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return fail(SD_EDEVICE, "hipGetDevice failed");
        RunKey key;
        std::memset(&key, 0, sizeof key);
        key.p = *p;
        key.n = n;
        key.x = x;
        key.force = force;
        key.v_prev = vp;
        key.dt = dt;
        key.integ = integrator;
        key.mode = integrator == SD_EULER ? 0 : 2;
        key.prec = precision;
        key.L = L;
        key.partial = partial;
        key.stage = stage;
        std::lock_guard<std::mutex> lk(g_rg_mu);
        RunGraph& g = g_rg[dev];
        if (!g.cap && hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking) != hipSuccess)
            return fail(SD_EDEVICE, "capture stream creation failed");
        if (!g.done && hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess)
            return fail(SD_EDEVICE, "event creation failed");
        if (!g.exec || !(g.key == key)) {
            drop_run_graph(g);
            if (hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return fail(SD_EDEVICE, "hipStreamBeginCapture failed");
            sd_status cst = SD_OK;
            for (int k = 0; k < RUN_CHUNK && !cst; ++k)   // step index 1: never the AB2 start
                cst = step_impl(p, n, x, force, vp, nullptr, dt, 1, integrator, precision, stage,
                                k > 0, k + 1 < RUN_CHUNK, (double*)partial, L, g.cap);
            hipGraph_t graph = nullptr;
            const hipError_t e2 = hipStreamEndCapture(g.cap, &graph);
            if (cst || e2 != hipSuccess || !graph) {
                if (graph) (void)hipGraphDestroy(graph);
                return cst ? cst : fail(SD_EDEVICE, "graph capture failed: %s", hipGetErrorString(e2));
            }
            hipGraphExec_t exec = nullptr;
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return fail(SD_EDEVICE, "hipGraphInstantiate failed");
            }
            g.graph = graph;
            g.exec = exec;
            g.key = key;
        }
        for (; done + RUN_CHUNK <= steps; done += RUN_CHUNK)
            if (hipGraphLaunch(g.exec, hs) != hipSuccess)
                return fail(SD_EDEVICE, "hipGraphLaunch failed");
        if (hipEventRecord(g.done, hs) != hipSuccess) return fail(SD_EDEVICE, "event record failed");
    }
    for (int64_t s = done; s < steps; ++s) {
        if ((st = step_impl(p, n, x, force, vp, nullptr, dt, step0 + s, integrator, precision, stage,
                            s > done, s + 1 < steps, (double*)partial, L, hs)))
            return st;
        if (x_checkpoints && (s + 1) % checkpoint_every == 0) {
            double* dst = x_checkpoints + 3 * (size_t)n * (size_t)((s + 1) / checkpoint_every);
            if (hipMemcpyAsync(dst, x, frame, hipMemcpyDeviceToDevice, hs) != hipSuccess)
                return fail(SD_EDEVICE, "checkpoint copy failed");
        }
    }
    return SD_OK;
}

sd_status sd_pack(int64_t n, const double* v, void* out, int32_t precision, void* stream)
{
    sd_status st;
    if ((st = check_n(n)) || (st = check_precision(precision))) return st;
    if ((st = check_ptr(v, 8, "v")) || (st = check_ptr(out, vec4_align(precision), "out")))
        return st;
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e = precision == SD_FP64 ? launch_pack_f64(v, (double4*)out, (int)n, hs)
                                        : launch_pack_f32(v, (float4*)out, (int)n, hs);
    if (e != hipSuccess) return fail(SD_EDEVICE, "pack launch: %s", hipGetErrorString(e));
    return SD_OK;
}

sd_status sd_mean_vector(int64_t n, const double* v, double* out, void* stream)
{
    sd_status st;
    if ((st = check_n(n)) || (st = check_ptr(v, 8, "v")) || (st = check_ptr(out, 8, "out")))
        return st;
    void* part = nullptr;
    if ((st = ws_get(WS_MEAN, 3 * (size_t)mean_groups(n) * sizeof(double), &part))) return st;
    hipError_t e = launch_mean_vector(v, n, out, (double*)part, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SD_EDEVICE, "mean launch: %s", hipGetErrorString(e));
    return SD_OK;
}

sd_status sd_premise_counts(int64_t* sub2a, int64_t* coincident, int32_t reset, void* stream)
{
    hipError_t e = premise_counts(sub2a, coincident, reset != 0, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SD_EDEVICE, "premise counts: %s", hipGetErrorString(e));
    return SD_OK;
}

sd_status sd_set_kernel_config(int32_t precision, const sd_kernel_config* cfg)
{
    sd_status st;
    if ((st = check_precision(precision))) return st;
    if (cfg && (st = check_config(precision, *cfg))) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cfg[precision].forced = cfg != nullptr;
    if (cfg) g_cfg[precision].forced_cfg = *cfg;
    return SD_OK;
}

sd_status sd_autotune_clear(int32_t precision)
{
    sd_status st;
    if ((st = check_precision(precision))) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cfg[precision].tuned.clear();
    return SD_OK;
}

sd_status sd_get_kernel_config(int32_t precision, int64_t n, sd_kernel_config* out)
{
    sd_status st;
    if ((st = check_precision(precision)) || (st = check_n(n))) return st;
    if (!out) return fail(SD_EINVAL, "out is NULL");
    *out = choose_config(precision, n);
    return SD_OK;
}

sd_status sd_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof.on = on != 0;
    return SD_OK;
}

sd_status sd_profile_read(int64_t* launches, double* total_ms)
{
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pend;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        pend.swap(g_prof.pending);
    }
    sd_status st = SD_OK;
    int64_t cnt = 0;
    double ms = 0.0;
    std::vector<float> times;
    for (auto& ab : pend) {
        float t = 0.0f;
        if (hipEventSynchronize(ab.second) != hipSuccess ||
            hipEventElapsedTime(&t, ab.first, ab.second) != hipSuccess)
            st = fail(SD_EDEVICE, "profiling event query failed");
        else {
            ms += t;
            ++cnt;
            times.push_back(t);
        }
        (void)hipEventDestroy(ab.first);
        (void)hipEventDestroy(ab.second);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof.launches += cnt;
    g_prof.total_ms += ms;
    for (float t : times)
        if (g_prof.times.size() < PROF_KEEP) g_prof.times.push_back(t);
    if (launches) *launches = g_prof.launches;
    if (total_ms) *total_ms = g_prof.total_ms;
    return st;
}

sd_status sd_profile_reset(void)
{
    int64_t l;
    double t;
    sd_profile_read(&l, &t);
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof.launches = 0;
    g_prof.total_ms = 0.0;
    g_prof.times.clear();
    return SD_OK;
}

sd_status sd_profile_times(float* ms, int64_t cap, int64_t* count)
{
    if (cap < 0) return fail(SD_EINVAL, "cap must be >= 0");
    if (cap > 0 && !ms) return fail(SD_EINVAL, "ms is NULL");
    sd_status st = sd_profile_read(nullptr, nullptr);
    std::lock_guard<std::mutex> lk(g_mu);
    const int64_t have = (int64_t)g_prof.times.size();
    for (int64_t i = 0; i < std::min(have, cap); ++i) ms[i] = g_prof.times[i];
    if (count) *count = have;
    return st;
}

sd_status sd_set_graph_mode(int32_t mode)
{
    if (mode < 0 || mode > 2) return fail(SD_EINVAL, "graph mode must be 0, 1 or 2");
    g_graph_mode = mode;
    return SD_OK;
}

sd_status sd_release(void)
{
    batch_release_graphs();
    run_graphs_release();
    return ws_release_all();
}

const char* sd_status_string(int32_t s)
{
    switch (s) {
    case SD_OK: return "SD_OK";
    case SD_EINVAL: return "SD_EINVAL: invalid argument";
    case SD_EALIGN: return "SD_EALIGN: misaligned pointer";
    case SD_ENOMEM: return "SD_ENOMEM: out of device memory";
    case SD_EDEVICE: return "SD_EDEVICE: HIP runtime or launch error";
    case SD_EUNSUPPORTED: return "SD_EUNSUPPORTED: not implemented for these arguments";
    default: return "unknown sd_status";
    }
}

const char* sd_last_error(void)
{
    return g_last_error.c_str();
}

int32_t sd_version(void)
{
    return SD_VERSION;
}

}  // extern "C"
