// sd_host.h -- host-side helpers shared by the C-ABI translation units
// (argument checks, workspace, launch planning).  Not part of the C ABI.
#pragma once

#include "sd.h"
#include "sd_internal.h"

namespace sd {

// Largest particle count the kernels index with 32-bit integers.
constexpr int64_t MAX_N = (int64_t(1) << 30);

// Library-owned workspace slots (one buffer each per device).
enum {
    WS_PARTIAL = 0,   // split partials of the pair kernels
    WS_STAGE,         // FP32 / FP64 staged positions of the time loop
    WS_ADJ_PARTIAL,   // split partials of the adjoint kernel
    WS_ADJ_PACK,      // packed cotangent / force staging
    WS_ADJ_TRAJ,      // recomputed trajectory of one checkpoint segment
    WS_ADJ_LAM,       // adjoint state
    WS_ADJ_CKPT,      // checkpoints when the caller passes none
    WS_TUNE,          // autotuner scratch
    WS_LUB,           // lubrication cell list
    WS_LUB_F,         // lubrication-corrected forces of a step
    WS_QPOS,          // fixed-point positions of a product in a periodic box
    WS_CLUSTER,       // run records of the precision study
    WS_MEAN,          // partial sums of sd_mean_vector
    WS_COUNT
};

sd_status fail(sd_status st, const char* fmt, ...);
sd_status check_lub(const sd_lub* lub);
sd_status check_params(const sd_params* p);
// cubic box side of validated params (0 = free space)
inline double box_side(const sd_params* p) { return p->box[0]; }
// SD_EUNSUPPORTED for a periodic box (entry points without box support)
sd_status check_free_space(const sd_params* p, const char* what);
sd_status check_n(int64_t n);
sd_status check_precision(int32_t prec);
sd_status check_ptr(const void* ptr, size_t align, const char* name);
size_t vec4_align(int32_t prec);
int device_cus();
sd_status ws_get(int which, size_t bytes, void** out);

sd_kernel_config default_config(int32_t prec, int64_t n);
// Whether the j-side workspace of the pair-symmetric kernel (variant 2) for n
// particles in blocks of `block` stays within SYM_WORKSPACE_CAP bytes.
constexpr size_t SYM_WORKSPACE_CAP = (size_t)1 << 30;
// Smallest n for which the automatic configuration takes variant 2.
constexpr int64_t SYM_MIN_N = 16384;
bool sym_fits(int64_t n, int block);
sd_kernel_config choose_config(int32_t prec, int64_t n);
void set_tuned_config(int32_t prec, int64_t n, const sd_kernel_config& c);
sd_status check_config(int32_t prec, const sd_kernel_config& c);

PairConst pair_const(const sd_params* p);
PairLaunch plan_pair(int32_t prec, int64_t n);
size_t partial_bytes(const PairLaunch& L, int64_t n);
// vel (may be null): for the pair-symmetric kernel the product is finished
// here (the fold merges into vel; *merged is set), else the caller merges.
sd_status run_pair(const sd_params* p, int64_t n, const void* pos, const void* frc,
                   const double* x64, int32_t prec, double* partial, const PairLaunch& L,
                   hipStream_t st, double* vel = nullptr, bool* merged = nullptr);

void batch_release_graphs();
void run_graphs_release();

}  // namespace sd
