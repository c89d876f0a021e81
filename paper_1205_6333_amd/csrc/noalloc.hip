// noalloc.hip -- mobility_apply_noalloc: the product of mobility_apply
// (Eq. 7a) with all of its device scratch in one static device array, for
// callers that cannot allocate device memory.
//
// Scratch: `scratch`, SD_NOALLOC_SCRATCH_BYTES per device, held from the
// library's load until the process ends.  Host code never uses the array's
// name as an address: the device address is taken once per device with
// hipGetSymbolAddress (on the entry point's first call on that device) and
// kept in g_scratch.  A call enqueues, on its stream, the one-sided LDS-tiled
// pair kernel (variant 0) writing its j-split partial rows into the array
// (every row element is written, nothing needs clearing) and the merge that
// reads them; in a periodic box the fixed-point position records go first in
// the array.  Calls on one device share the array: calls that overlap in time
// on one device race.
#include "sd.h"
#include "sd_host.h"
#include "sd_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

namespace {

__device__ __align__(256) unsigned char scratch[SD_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch;   // device -> address of `scratch` there

sd_status scratch_of_current_device(unsigned char** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return sd::fail(SD_EDEVICE, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return SD_OK;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return sd::fail(SD_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    g_scratch[dev] = (unsigned char*)p;
    *out = (unsigned char*)p;
    return SD_OK;
}

}  // namespace

using namespace sd;

extern "C" sd_status mobility_apply_noalloc(const sd_params* p, int64_t n, const void* pos,
                                            const void* force, double* vel, int32_t precision,
                                            void* stream)
{
    sd_status st;
    if ((st = check_params(p)) || (st = check_n(n)) || (st = check_precision(precision))) return st;
    const size_t al = vec4_align(precision);
    if ((st = check_ptr(pos, al, "pos")) || (st = check_ptr(force, al, "force")) ||
        (st = check_ptr(vel, 8, "vel")))
        return st;
    const bool box = box_side(p) > 0.0 && precision != SD_FP64;
    const size_t row = 3 * (size_t)n * sizeof(double);     // one partial row
    const size_t qbytes = box ? (((size_t)n * 16 + 255) & ~(size_t)255) : 0;
    if (qbytes + row > SD_NOALLOC_SCRATCH_BYTES)
        return fail(SD_EINVAL, "n = %lld exceeds the %u-byte scratch of mobility_apply_noalloc "
                               "(at most %zu particles%s)",
                    (long long)n, (unsigned)SD_NOALLOC_SCRATCH_BYTES,
                    (size_t)SD_NOALLOC_SCRATCH_BYTES / (box ? 40 : 24),
                    box ? " in a periodic box" : "");
    unsigned char* base = nullptr;
    if ((st = scratch_of_current_device(&base))) return st;
    // the automatic shape of the one-sided kernel, with no more split rows
    // than the scratch holds
    sd_kernel_config c = default_config(precision, n);
    const int64_t fit = (int64_t)((SD_NOALLOC_SCRATCH_BYTES - qbytes) / row);
    const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(c.splits, fit));
    PairLaunch L = shape_pair_launch((int)n, 0, c.block, splits, 1, 0);
    L.acc = (precision == SD_FP32_KAHAN) ? (c.block >= 128 ? 8 : 4) : 0;
    double* partial = (double*)(base + qbytes);
    hipStream_t hs = (hipStream_t)stream;
    const PairConst pc = pair_const(p);
    hipError_t e = hipSuccess;
    const void* pos_k = pos;
    if (box) {
        e = launch_stage_q_from_f32((const float4*)pos, (float4*)base, (int)n, box_side(p), hs);
        pos_k = base;
    }
    const double mu0 = 1.0 / (6.0 * M_PI * p->eta * p->a);
    if (e == hipSuccess) {
        if (precision == SD_FP64) {
            e = launch_pair_f64(L, p->tensor, (const double4*)pos_k, (const double4*)force,
                                (int)n, pc, partial, hs);
            if (e == hipSuccess)
                e = launch_merge_f64(partial, L.splits, (int)n, (const double4*)force, mu0, vel,
                                     hs);
        } else {
            e = launch_pair_f32(L, p->tensor, L.acc, (const float4*)pos_k, (const float4*)force,
                                nullptr, (int)n, pc, partial, hs);
            if (e == hipSuccess)
                e = launch_merge_f32(partial, L.splits, (int)n, (const float4*)force, mu0, vel, hs);
        }
    }
    if (e != hipSuccess) return fail(SD_EDEVICE, "launch: %s", hipGetErrorString(e));
    return SD_OK;
}
