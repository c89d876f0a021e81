// sd_internal.h -- declarations shared by the HIP translation units of the
// library (kernel launchers, constants, workspace).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sd {

enum { T_RPY = 0, T_OSEEN = 1 };

// Pair-tensor constants in the form the kernels use.
//
// Both tensors are written as T(r) = alpha [A'(r) I + Bt'(r) r r] with
// alpha = 1/(8 pi eta) (= mu0 * 3a/4):
//   Rotne-Prager, Eq. (7b):  A' = 1/r + gamma/r^3,  Bt' = (1 - 3 gamma/r^2)/r^3,
//                            gamma = 2a^2/3
//   Oseen, Eq. (4):          A' = 1/r,             Bt' = 1/r^3
// so the FP32 fast path accumulates A' F + Bt' (d.F) d and the product with
// alpha is taken once per particle, in FP64.  Pairs with r^2 < thr2 (near
// contact, overlap, coincidence, self) skip the fast path and are evaluated in
// FP64 from the same definitions.
//
// Periodic cubic box of side Lb (nearest image, footnote of Sec. 3.1): the
// FP32 path stages positions as 32-bit fixed-point fractions of the box,
// q = x 2^32 / Lb mod 2^32, so that the wrapped integer difference
// q_i - q_j (two's complement) is exactly the nearest-image difference in
// units of s = Lb / 2^32 (a difference of exactly Lb/2 becomes -Lb/2).  With
// d = s e the pair term is (alpha / s) [A'(e; gamma/s^2) F + Bt'(e; gamma/s^2)
// (e.F) e], so the FP32 constants below are the scaled ones and the scale is
// folded into alpha_sum.  The FP64 path folds d -= Lb rint(d / Lb).
struct PairConst {
    float gamma_f;       // 2a^2/3 (RPY) or 0 (Oseen); / s^2 when periodic
    float m3gamma_f;     // -3 gamma_f
    float thr2_f;        // near threshold on r^2, FP32 (/ s^2 when periodic)
    int overlap;         // 1: overlap form for r < 2a (RPY only)
    double thr2_d;       // near threshold on r^2, FP64 (physical units)
    double alpha;        // 1/(8 pi eta)
    double alpha_sum;    // factor of the FP32 sums: alpha, or alpha / s when periodic
    double gamma;        // 2a^2/3 (RPY) or 0 (Oseen)
    double mu0;          // 1/(6 pi eta a)
    double a;
    double box;          // cubic box side Lb, 0 = free space
    double ibox;         // 1 / Lb (0 in free space)
    double s_q;          // fixed-point unit Lb / 2^32 (0 in free space)
};

// Nearest image of a difference vector, FP64 (round-half-even of d / Lb).
__host__ __device__ inline void nearest_image_d(const PairConst& pc, double& d0, double& d1,
                                                double& d2)
{
    if (pc.box > 0.0) {
        d0 -= pc.box * rint(d0 / pc.box);
        d1 -= pc.box * rint(d1 / pc.box);
        d2 -= pc.box * rint(d2 / pc.box);
    }
}

// Relative widening of the near threshold: pairs with r^2 < (2a)^2 (1 + NEAR_EPS)
// are evaluated in FP64.
constexpr double NEAR_EPS = 1e-3;

// box: cubic box side (0 = free space).
PairConst make_pair_const(double a, double eta, int tensor, int overlap, double box);

struct PairLaunch {
    int variant;   // 0 LDS tiles, 1 scalar-cache j stream, 2 pair symmetry (FP32 only)
    int block;     // threads per work-group
    int splits;    // number of partial rows written (variants 0/1: j-range splits)
    int jchunk;    // variants 0/1: particles j per split (multiple of block);
                   // variant 2: the requested split count the schedule was cut from
    int ilp;       // i per lane
    int acc;       // FP32 accumulation: 0 plain, k = Kahan per k terms
    int cus;       // variant 2: compute units the schedule was cut for
};

// Shape the launch for n particles from a requested configuration on a device
// with `cus` compute units.
PairLaunch shape_pair_launch(int n, int variant, int block, int splits, int ilp, int cus);

// Block schedule of variant 2 (each pair of distinct blocks once, see
// k_pair_f32_sym): nb blocks of `block` particles; i-block I takes the h
// blocks after it (mod nb) and, when nb is even (extra = 1), block I + nb/2
// if I < nb/2; that virtual j range (at most lmax positions, lmax / SYM_TJ
// tiles) is cut into isplits splits, split k covering tiles
// [off[k], off[k+1]).  The splits shrink towards the end (see sym_shape), so
// that the last work-groups of a launch are short.  Partial rows: isplits
// symmetric splits, one row of the one-sided diagonal blocks, one row of the
// folded j side and the near pairs, so PairLaunch.splits = isplits + 2.
// After the rows (256-byte aligned) the workspace holds the FP32 j-side
// partials, 3 * nb * lmax floats, then (256-byte aligned) the near-pair
// records: one 16-byte entry per wave row and tile of the virtual range, then
// one per wave row for its own block (see sym_flag_row in mobility.hip);
// every product rewrites every entry it reads.
constexpr int SYM_TJ = 128;          // j tile of the symmetric kernel
constexpr int SYM_MAX_SPLITS = 96;
// The particles of one wave and lane slot: SYM_RUN consecutive particles.
constexpr int SYM_RUN = 64;
struct SymShape {
    int nb, h, extra, lmax, isplits;
    int nt;   // tiles of SYM_TJ in the longest virtual j range (lmax / SYM_TJ)
    int off[SYM_MAX_SPLITS + 1];
};
// splits: the largest split covers about 1/splits of the range; slots:
// work-groups resident on the device at once.
SymShape sym_shape(int n, int block, int splits, int slots);
// resident work-groups of the symmetric kernel with `block` lanes on `cus` CUs
int sym_slots(int block, int cus);
SymShape sym_shape_of(const PairLaunch& L, int n);
size_t sym_jpart_floats(const SymShape& sh);
size_t sym_jpart_offset(const PairLaunch& L, int64_t n);
size_t sym_flags_offset(const PairLaunch& L, int64_t n);
size_t sym_workspace_bytes(const PairLaunch& L, int64_t n);
// near flags: (nb * block / SYM_RUN) x nt bytes, then nb * block / SYM_RUN
size_t sym_flags_bytes(const SymShape& sh, int block);

// Pair kernels: partial[(s*3 + k)*n + i] = sum over split s of the pair terms
// (self excluded), FP64 output.
// x64 (f64[3n], may be null): FP64 positions used for near pairs.
// With pc.box > 0 the FP32 kernel reads fixed-point positions (uint4 bits in
// the float4 records, see PairConst) and the FP64 kernel folds differences.
hipError_t launch_pair_f32(const PairLaunch& L, int tensor, int acc, const float4* pos,
                           const float4* frc, const double* x64, int n, const PairConst& pc,
                           double* partial, hipStream_t st);
hipError_t launch_pair_f64(const PairLaunch& L, int tensor, const double4* pos, const double4* frc,
                           int n, const PairConst& pc, double* partial, hipStream_t st);
// Variant 2 only (a no-op otherwise): the last partial row, from the j-side
// partials and the near-pair flags the pair kernel left in the workspace.
// pos/frc: the records the pair kernel read; x64 as for launch_pair_f32.
// Enqueue after the pair kernel, before anything reads the partial rows.
// With vel (f64[3n]) given, the fold also does the merge: vel = mu0 F + the
// split rows in order + the folded row, the sum k_merge forms, bit for bit,
// and the folded row is not written.
hipError_t launch_pair_fold(const PairLaunch& L, int tensor, const float4* pos, const float4* frc,
                            const double* x64, int n, const PairConst& pc, double* partial,
                            hipStream_t st, double mu0 = 0.0, double* vel = nullptr);

// v_i = mu0 F_i + sum_s partial_s (fixed order).
// Read the current device's counts of pairs with 0 < r < 2a and r = 0 met by
// the product kernels (stream-ordered; synchronises st), zeroing them if reset.
hipError_t premise_counts(int64_t* sub2a, int64_t* coincident, bool reset, hipStream_t st);
hipError_t launch_merge_f32(const double* partial, int splits, int n, const float4* frc, double mu0,
                            double* vel, hipStream_t st);
hipError_t launch_merge_f64(const double* partial, int splits, int n, const double4* frc,
                            double mu0, double* vel, hipStream_t st);

// Time loop helpers.  box > 0: the FP32 stage is the fixed-point form of a
// periodic box of that side (see PairConst); the FP64 stage is unchanged.
hipError_t launch_stage_f32(const double* x, float4* pos, int n, double box, hipStream_t st);
hipError_t launch_stage_f64(const double* x, double4* pos, int n, hipStream_t st);
// fixed-point form of FP32 position records (mobility product in a box)
hipError_t launch_stage_q_from_f32(const float4* pos, float4* q, int n, double box,
                                   hipStream_t st);
// mode: 0 Euler, 1 AB2 start (Euler + store v_prev), 2 AB2
hipError_t launch_merge_integrate_f32(const double* partial, int splits, int n, const float4* frc,
                                      double mu0, double* x, double* v_prev, double* v_out,
                                      double dt, int mode, float4* pos_next, double box,
                                      hipStream_t st);
hipError_t launch_merge_integrate_f64(const double* partial, int splits, int n, const double4* frc,
                                      double mu0, double* x, double* v_prev, double* v_out,
                                      double dt, int mode, double4* pos_next, hipStream_t st);

// Adjoint pair kernels: partial[(s*3+k)*n + i] = position gradient terms,
// partial_f[...] = pair part of (M lam)_i.
hipError_t launch_adjoint_f32(const PairLaunch& L, int tensor, const float4* pos, const float4* frc,
                              const float4* lam, const double* x64, int n, const PairConst& pc,
                              double* partial, double* partial_f, hipStream_t st);
hipError_t launch_adjoint_f64(const PairLaunch& L, int tensor, const double4* pos,
                              const double4* frc, const double4* lam, int n, const PairConst& pc,
                              double* partial, double* partial_f, hipStream_t st);
// out[3i+k] = sum_s partial (no self term); accumulate != 0 adds scale*sum to out.
hipError_t launch_sum_partials(const double* partial, int splits, int n, double* out, double scale,
                               int accumulate, hipStream_t st);
// f64[3n] -> f32x4 / f64x4 (w = 0)
hipError_t launch_pack_f32(const double* v, float4* out, int n, hipStream_t st);
hipError_t launch_pack_f64(const double* v, double4* out, int n, hipStream_t st);
// y[k] += s * x[k], k < m
hipError_t launch_axpy(double s, const double* x, double* y, int64_t m, hipStream_t st);

// Batched clusters.
struct BatchDev {
    const int64_t* offsets;   // device, C+1
    const int32_t* order;     // device, C: processing order (longest first)
    int32_t* counter;         // device, 1: work-queue head
    int n_clusters;
    int max_size;
    int wg;                   // lanes per work-group: 128, 256 or 512
};
hipError_t launch_batched_run(const BatchDev& b, int tensor, int precision, const PairConst& pc,
                              double* x, const void* frc, double dt, int steps, int integrator,
                              int n_workgroups, hipStream_t st);
hipError_t launch_batched_apply(const BatchDev& b, int tensor, int precision, const PairConst& pc,
                                const void* pos, const void* frc, double* vel, int n_workgroups,
                                hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int32_t value, int count, hipStream_t st);
// out = (1/n) sum_i v_i (deterministic); partial: f64[3 mean_groups(n)] scratch
int64_t mean_groups(int64_t n);
hipError_t launch_mean_vector(const double* v, int64_t n, double* out, double* partial,
                              hipStream_t st);
size_t batched_lds_bytes(int max_size, int precision, int integrator, int wg);

}  // namespace sd
