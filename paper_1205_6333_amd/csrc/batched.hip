// batched.hip -- many independent clusters, each a free-space suspension of
// its own (the mobility product of Eq. 7a restricted to a cluster, advanced by
// the step loop of Sec. 3.1), in ONE persistent kernel launch.
//
// Each work-group of WG lanes (128, 256 or 512, chosen per plan, e.g. by the
// autotuner) pulls cluster ids from a device work queue (an atomic counter
// over a longest-first order prepared on the host), loads the cluster into LDS
// (FP64 master positions, forces, FP32 staged positions) and runs all time
// steps without leaving the kernel: clusters never interact, so no grid-wide
// synchronisation is needed.  Clusters of nc <= WG particles have the j range
// of each particle cut into Q pieces, and the nc Q (piece, particle) items
// dealt round-robin to the lanes (Q chosen per cluster so that the longest
// lane's share is smallest); the Q partial velocities of a particle are
// combined in LDS in a fixed order.  Larger clusters (up to
// SD_BATCH_MAX_CLUSTER) give each lane ceil(nc / WG) particles.
#include "pair_terms.h"
#include "sd.h"
#include "sd_host.h"
#include "sd_internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>
#include <cstdio>
#include <string>
#include <vector>

namespace sd {


// LDS layout of one work-group (every segment 32-byte aligned):
//   xs  2 x f64[3M]   FP64 positions of the cluster, double-buffered: a step
//                     reads one copy and writes the next positions to the other
//   fs  f32x4[M] or f64x4[M]   forces
//   pf  2 x f32x4[M]  FP32 staged positions (FP32 precisions), double-buffered
//   vp  f64[3M]   previous velocities (AB2)
//   red f64[3*max(B_ITEMS_PER_LANE WG, M)] partial velocities of the
//                 (piece, particle) items, or the velocities of the cluster
//                 (more particles than lanes)
// partial sums per lane of the work-group (see b_pieces)
constexpr int B_ITEMS_PER_LANE = 2;

struct LdsLayout {
    size_t xs1, fs, pf, pf1, vp, red, total;
};

__host__ __device__ inline size_t lds_round(size_t b) { return (b + 31) & ~(size_t)31; }

__host__ __device__ inline LdsLayout lds_layout(int max_size, int precision, int integrator,
                                                int wg)
{
    const size_t M = (size_t)max_size;
    LdsLayout L;
    size_t o = lds_round(M * 3 * sizeof(double));
    L.xs1 = o;
    o += lds_round(M * 3 * sizeof(double));
    L.fs = o;
    o += lds_round(M * (precision == SD_FP64 ? sizeof(double4) : sizeof(float4)));
    L.pf = o;
    if (precision != SD_FP64) o += lds_round(M * sizeof(float4));
    L.pf1 = o;
    if (precision != SD_FP64) o += lds_round(M * sizeof(float4));
    L.vp = o;
    if (integrator == SD_AB2) o += lds_round(M * 3 * sizeof(double));
    L.red = o;
    const size_t items = (size_t)B_ITEMS_PER_LANE * wg;
    o += lds_round((items > M ? items : M) * 3 * sizeof(double));
    L.total = o;
    return L;
}

size_t batched_lds_bytes(int max_size, int precision, int integrator, int wg)
{
    return lds_layout(max_size, precision, integrator, wg).total;
}


// Velocity (pair part, physical units, self term excluded) of particle i from
// the particles j0 <= j < j1 of the cluster held in LDS.
// PREC: SD_FP32_KAHAN (Kahan once per block of 16 terms), SD_FP32_PLAIN, SD_FP64.
template <int TENSOR, int PREC>
__device__ __forceinline__ void b_velocity(int i, int j0, int j1, const double* xs,
                                           const void* fsv, const float4* pf, const PairConst& pc,
                                           double* v)
{
    double nv[3] = { 0.0, 0.0, 0.0 };
    if (PREC == SD_FP64) {
        const double4* fs = (const double4*)fsv;
        const double xi0 = xs[3 * i], xi1 = xs[3 * i + 1], xi2 = xs[3 * i + 2];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int j = j0; j < j1; ++j) {
            const double dx = xi0 - xs[3 * j], dy = xi1 - xs[3 * j + 1], dz = xi2 - xs[3 * j + 2];
            const double4 fj = fs[j];
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            if (r2 < pc.thr2_d) {
                if (j != i) near_term<TENSOR>(pc, dx, dy, dz, fj.x, fj.y, fj.z, nv[0], nv[1], nv[2]);
                continue;
            }
            const double rinv = rsqrt(r2);
            const double rinv2 = rinv * rinv, rinv3 = rinv2 * rinv;
            double A = rinv, Bt = rinv3;
            if (TENSOR == T_RPY) {
                A = fma(pc.gamma, rinv3, rinv);
                Bt = rinv3 * fma(-3.0 * pc.gamma, rinv2, 1.0);
            }
            const double sB = Bt * fma(dx, fj.x, fma(dy, fj.y, dz * fj.z));
            a0 = fma(A, fj.x, fma(sB, dx, a0));
            a1 = fma(A, fj.y, fma(sB, dy, a1));
            a2 = fma(A, fj.z, fma(sB, dz, a2));
        }
        v[0] = pc.alpha * a0 + nv[0];
        v[1] = pc.alpha * a1 + nv[1];
        v[2] = pc.alpha * a2 + nv[2];
        return;
    }
    constexpr bool KAHAN = PREC == SD_FP32_KAHAN;
    const float4* fs = (const float4*)fsv;
    const float4 pi = pf[i];
    // the constants in VGPRs: a VALU instruction with an SGPR operand issues
    // at half rate on gfx950
    float gamma = pc.gamma_f, m3g = pc.m3gamma_f, thr2 = pc.thr2_f;
    asm volatile("" : "+v"(gamma), "+v"(m3g), "+v"(thr2));
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    // four consecutive j into the running block sum y: one near test per four
    // (pairs below the threshold are evaluated in FP64 from the FP64 positions
    // and get r^2 = +inf, an exact zero, in the FP32 code)
    auto group4 = [&](int j, float& y0, float& y1, float& y2) {
        // one group's data live at a time (overlapping four groups of a block
        // doubles the register count and halves the resident waves)
        __builtin_amdgcn_sched_barrier(0);
        float4 pj[4], fj[4];
        float dx[4], dy[4], dz[4], r2[4];
        float rmin = 0.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pj[u] = pf[j + u];
            fj[u] = fs[j + u];
            dx[u] = pi.x - pj[u].x;
            dy[u] = pi.y - pj[u].y;
            dz[u] = pi.z - pj[u].z;
            r2[u] = fmaf(dx[u], dx[u], fmaf(dy[u], dy[u], dz[u] * dz[u]));
            rmin = u == 0 ? r2[0] : fminf(rmin, r2[u]);
        }
        if (__builtin_amdgcn_ballot_w64(rmin < thr2) != 0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int jj = j + u;
                if (r2[u] < thr2 && jj != i)
                    near_term<TENSOR>(pc, xs[3 * i] - xs[3 * jj], xs[3 * i + 1] - xs[3 * jj + 1],
                                      xs[3 * i + 2] - xs[3 * jj + 2], fj[u].x, fj[u].y, fj[u].z,
                                      nv[0], nv[1], nv[2]);
                r2[u] = (r2[u] < thr2) ? __builtin_inff() : r2[u];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float rinv = __builtin_amdgcn_rsqf(r2[u]);
            const float rinv2 = rinv * rinv, rinv3 = rinv2 * rinv;
            float A = rinv, Bt = rinv3;
            if (TENSOR == T_RPY) {
                A = fmaf(gamma, rinv3, rinv);
                Bt = rinv3 * fmaf(m3g, rinv2, 1.0f);
            }
            const float sB = Bt * fmaf(dx[u], fj[u].x, fmaf(dy[u], fj[u].y, dz[u] * fj[u].z));
            y0 = fmaf(A, fj[u].x, fmaf(sB, dx[u], y0));
            y1 = fmaf(A, fj[u].y, fmaf(sB, dy[u], y1));
            y2 = fmaf(A, fj[u].z, fmaf(sB, dz[u], y2));
        }
    };
    // a block sum seeded with the negated compensation, then one compensated add
    auto commit = [&](float y0, float y1, float y2) {
        if (KAHAN) {
            const float t0 = s0 + y0, t1 = s1 + y1, t2 = s2 + y2;
            c0 = (t0 - s0) - y0;
            c1 = (t1 - s1) - y1;
            c2 = (t2 - s2) - y2;
            s0 = t0;
            s1 = t1;
            s2 = t2;
        } else {
            s0 = y0;
            s1 = y1;
            s2 = y2;
        }
    };
    int j = j0;
    for (; j + 16 <= j1; j += 16) {   // blocks of 16 terms
        float y0 = KAHAN ? -c0 : s0, y1 = KAHAN ? -c1 : s1, y2 = KAHAN ? -c2 : s2;
#pragma unroll 1
        for (int g = 0; g < 16; g += 4) group4(j + g, y0, y1, y2);
        commit(y0, y1, y2);
    }
    for (; j + 4 <= j1; j += 4) {     // then blocks of 4
        float y0 = KAHAN ? -c0 : s0, y1 = KAHAN ? -c1 : s1, y2 = KAHAN ? -c2 : s2;
        group4(j, y0, y1, y2);
        commit(y0, y1, y2);
    }
    for (; j < j1; ++j) {             // and single terms
        const float4 pj = pf[j];
        const float4 fj = fs[j];
        const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        if (r2 < thr2) {
            if (j != i)
                near_term<TENSOR>(pc, xs[3 * i] - xs[3 * j], xs[3 * i + 1] - xs[3 * j + 1],
                                  xs[3 * i + 2] - xs[3 * j + 2], fj.x, fj.y, fj.z, nv[0], nv[1],
                                  nv[2]);
            continue;
        }
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float rinv2 = rinv * rinv, rinv3 = rinv2 * rinv;
        float A = rinv, Bt = rinv3;
        if (TENSOR == T_RPY) {
            A = fmaf(gamma, rinv3, rinv);
            Bt = rinv3 * fmaf(m3g, rinv2, 1.0f);
        }
        const float sB = Bt * fmaf(dx, fj.x, fmaf(dy, fj.y, dz * fj.z));
        const float y0 = fmaf(A, fj.x, fmaf(sB, dx, KAHAN ? -c0 : s0));
        const float y1 = fmaf(A, fj.y, fmaf(sB, dy, KAHAN ? -c1 : s1));
        const float y2 = fmaf(A, fj.z, fmaf(sB, dz, KAHAN ? -c2 : s2));
        commit(y0, y1, y2);
    }
    v[0] = pc.alpha * ((double)s0 - (double)c0) + nv[0];
    v[1] = pc.alpha * ((double)s1 - (double)c1) + nv[1];
    v[2] = pc.alpha * ((double)s2 - (double)c2) + nv[2];
}

// Pieces per particle for a cluster of nc <= WG particles: the j range of each
// particle is cut into Q pieces of ceil(nc / Q), and the nc Q (piece,
// particle) items are dealt round-robin to the WG lanes.  Q minimises the
// longest lane's share, ceil(nc Q / WG) ceil(nc / Q), with at most
// B_ITEMS_PER_LANE WG items (the LDS of the partial sums); ties take the
// smaller Q.

__host__ __device__ inline int b_pieces(int nc, int wg)
{
    int best_q = 1;
    long best = -1;
    for (int q = 1; q <= nc && nc * q <= B_ITEMS_PER_LANE * wg; ++q) {
        const long w = (long)((nc * q + wg - 1) / wg) * (long)((nc + q - 1) / q);
        if (best < 0 || w < best) {
            best = w;
            best_q = q;
        }
    }
    return best_q;
}

// RUN: `steps` steps per cluster, positions written back to x.
// APPLY (steps < 0): one product, velocities written to vel.
// Per step: every lane computes its share of the velocities from one copy of
// the positions, the owners of the particles write the next positions to the
// other copy, and one barrier ends the step (two when Q > 1: the partial
// velocities of a particle are summed by its owner after a barrier).
template <int TENSOR, int PREC, int INTEG, int WG>
__global__ void __launch_bounds__(WG)
k_batched(BatchDev b, PairConst pc, double* __restrict__ x, const void* __restrict__ frc,
          double* __restrict__ vel, double dt, int steps)
{
    constexpr int BB = WG;
    extern __shared__ __align__(32) unsigned char lds[];
    const LdsLayout lay = lds_layout(b.max_size, PREC, INTEG, WG);
    double* const xs0 = (double*)lds;
    double* const xs1 = (double*)(lds + lay.xs1);
    void* fs = lds + lay.fs;
    float4* const pf0 = (PREC != SD_FP64) ? (float4*)(lds + lay.pf) : nullptr;
    float4* const pf1 = (PREC != SD_FP64) ? (float4*)(lds + lay.pf1) : nullptr;
    double* vp = (INTEG == SD_AB2) ? (double*)(lds + lay.vp) : nullptr;
    double* red = (double*)(lds + lay.red);
    __shared__ int s_item;
    const int t = threadIdx.x;

    for (;;) {
        __syncthreads();  // the previous cluster's write-back has read every copy
        if (t == 0) s_item = atomicAdd(b.counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= b.n_clusters) break;  // every work-group exits once the queue is empty
        const int c = b.order[item];
        const int64_t off = b.offsets[c];
        const int nc = (int)(b.offsets[c + 1] - off);
        if (nc <= 0) continue;
        for (int k = t; k < nc; k += BB) {
            const size_t g = (size_t)(off + k);
            const double x0 = x[3 * g], x1 = x[3 * g + 1], x2 = x[3 * g + 2];
            xs0[3 * k] = x0;
            xs0[3 * k + 1] = x1;
            xs0[3 * k + 2] = x2;
            if (PREC != SD_FP64) pf0[k] = make_float4((float)x0, (float)x1, (float)x2, 0.0f);
            if (PREC == SD_FP64)
                ((double4*)fs)[k] = ((const double4*)frc)[g];
            else
                ((float4*)fs)[k] = ((const float4*)frc)[g];
        }
        __syncthreads();
        // nc <= BB: Q pieces per particle, items q nc + i dealt round-robin
        // (consecutive lanes take consecutive particles of one piece, so a
        // wave's j reads are LDS broadcasts); larger clusters: rows of BB
        // particles per lane
        const int Q = nc <= BB ? b_pieces(nc, BB) : 1;
        const int C = (nc + Q - 1) / Q;
        const int rows = nc <= BB ? 1 : (nc + BB - 1) / BB;
        const int nsteps = steps < 0 ? 1 : steps;
        // current copy (read this step) and next copy (written this step)
        double* xs = xs0;
        double* xn = xs1;
        float4* pf = pf0;
        float4* pn = pf1;
        for (int st = 0; st < nsteps; ++st) {
            // velocities (pair part) of the particles this lane owns
            double v[3] = { 0.0, 0.0, 0.0 };  // rows == 1: the owner's velocity
            if (rows == 1 && Q == 1) {
                if (t < nc) b_velocity<TENSOR, PREC>(t, 0, nc, xs, fs, pf, pc, v);
            } else if (rows == 1) {
                for (int it = t; it < nc * Q; it += BB) {
                    const int q = it / nc, i = it - q * nc;
                    const int j0 = q * C, j1 = min(j0 + C, nc);
                    double w[3];
                    b_velocity<TENSOR, PREC>(i, j0, j1, xs, fs, pf, pc, w);
                    red[3 * it] = w[0];
                    red[3 * it + 1] = w[1];
                    red[3 * it + 2] = w[2];
                }
                __syncthreads();
                if (t < nc)
                    for (int q = 0; q < Q; ++q) {   // the pieces in order
                        v[0] += red[3 * (q * nc + t)];
                        v[1] += red[3 * (q * nc + t) + 1];
                        v[2] += red[3 * (q * nc + t) + 2];
                    }
            } else {
                // rows of BB particles per lane: velocities to this lane's slots
                for (int r = 0; r < rows; ++r) {
                    const int i = t + r * BB;
                    if (i >= nc) break;
                    double w[3];
                    b_velocity<TENSOR, PREC>(i, 0, nc, xs, fs, pf, pc, w);
                    red[3 * i] = w[0];
                    red[3 * i + 1] = w[1];
                    red[3 * i + 2] = w[2];
                }
            }
            // owners: velocity out (APPLY) or the next positions into the other copy
            for (int r = 0; r < rows; ++r) {
                const int i = t + r * BB;
                if (i >= nc) continue;
                const double w0 = rows == 1 ? v[0] : red[3 * i];
                const double w1 = rows == 1 ? v[1] : red[3 * i + 1];
                const double w2 = rows == 1 ? v[2] : red[3 * i + 2];
                double f0, f1, f2;
                if (PREC == SD_FP64) {
                    const double4 f = ((const double4*)fs)[i];
                    f0 = f.x; f1 = f.y; f2 = f.z;
                } else {
                    const float4 f = ((const float4*)fs)[i];
                    f0 = f.x; f1 = f.y; f2 = f.z;
                }
                const double vv[3] = { pc.mu0 * f0 + w0, pc.mu0 * f1 + w1, pc.mu0 * f2 + w2 };
                if (steps < 0) {
                    const size_t g = (size_t)(off + i);
                    vel[3 * g] = vv[0];
                    vel[3 * g + 1] = vv[1];
                    vel[3 * g + 2] = vv[2];
                    continue;
                }
                double xnew[3];
                for (int k = 0; k < 3; ++k) {
                    double inc = vv[k];
                    if (INTEG == SD_AB2) {
                        if (st > 0) inc = 1.5 * vv[k] - 0.5 * vp[3 * i + k];
                        vp[3 * i + k] = vv[k];
                    }
                    xnew[k] = xs[3 * i + k] + dt * inc;
                    xn[3 * i + k] = xnew[k];
                }
                if (PREC != SD_FP64)
                    pn[i] = make_float4((float)xnew[0], (float)xnew[1], (float)xnew[2], 0.0f);
            }
            __syncthreads();  // the next step reads the copy written above
            double* const tx = xs;
            xs = xn;
            xn = tx;
            float4* const tp = pf;
            pf = pn;
            pn = tp;
        }
        if (steps >= 0) {
            for (int k = t; k < nc; k += BB) {
                const size_t g = (size_t)(off + k);
                x[3 * g] = xs[3 * k];
                x[3 * g + 1] = xs[3 * k + 1];
                x[3 * g + 2] = xs[3 * k + 2];
            }
        }
    }
}

template <int TENSOR, int PREC, int INTEG, int WG>
static hipError_t launch_bw(const BatchDev& b, const PairConst& pc, double* x, const void* frc,
                            double* vel, double dt, int steps, int nwg, hipStream_t st)
{
    const size_t lds = batched_lds_bytes(b.max_size, PREC, INTEG, WG);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_batched<TENSOR, PREC, INTEG, WG>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_batched<TENSOR, PREC, INTEG, WG>), dim3(nwg), dim3(WG), lds, st, b, pc,
                       x, frc, vel, dt, steps);
    return hipGetLastError();
}

template <int TENSOR, int PREC, int INTEG>
static hipError_t launch_b(const BatchDev& b, const PairConst& pc, double* x, const void* frc,
                           double* vel, double dt, int steps, int nwg, hipStream_t st)
{
    switch (b.wg) {
    case 128: return launch_bw<TENSOR, PREC, INTEG, 128>(b, pc, x, frc, vel, dt, steps, nwg, st);
    case 256: return launch_bw<TENSOR, PREC, INTEG, 256>(b, pc, x, frc, vel, dt, steps, nwg, st);
    case 512: return launch_bw<TENSOR, PREC, INTEG, 512>(b, pc, x, frc, vel, dt, steps, nwg, st);
    }
    return hipErrorInvalidValue;
}

template <int TENSOR>
static hipError_t launch_bt(const BatchDev& b, int prec, int integ, const PairConst& pc, double* x,
                            const void* frc, double* vel, double dt, int steps, int nwg,
                            hipStream_t st)
{
    switch (prec * 2 + integ) {
    case SD_FP32_KAHAN * 2 + SD_EULER:
        return launch_b<TENSOR, SD_FP32_KAHAN, SD_EULER>(b, pc, x, frc, vel, dt, steps, nwg, st);
    case SD_FP32_KAHAN * 2 + SD_AB2:
        return launch_b<TENSOR, SD_FP32_KAHAN, SD_AB2>(b, pc, x, frc, vel, dt, steps, nwg, st);
    case SD_FP64 * 2 + SD_EULER:
        return launch_b<TENSOR, SD_FP64, SD_EULER>(b, pc, x, frc, vel, dt, steps, nwg, st);
    case SD_FP64 * 2 + SD_AB2:
        return launch_b<TENSOR, SD_FP64, SD_AB2>(b, pc, x, frc, vel, dt, steps, nwg, st);
    case SD_FP32_PLAIN * 2 + SD_EULER:
        return launch_b<TENSOR, SD_FP32_PLAIN, SD_EULER>(b, pc, x, frc, vel, dt, steps, nwg, st);
    case SD_FP32_PLAIN * 2 + SD_AB2:
        return launch_b<TENSOR, SD_FP32_PLAIN, SD_AB2>(b, pc, x, frc, vel, dt, steps, nwg, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batched_run(const BatchDev& b, int tensor, int precision, const PairConst& pc,
                              double* x, const void* frc, double dt, int steps, int integrator,
                              int n_workgroups, hipStream_t st)
{
    return tensor == T_OSEEN
               ? launch_bt<T_OSEEN>(b, precision, integrator, pc, x, frc, nullptr, dt, steps,
                                    n_workgroups, st)
               : launch_bt<T_RPY>(b, precision, integrator, pc, x, frc, nullptr, dt, steps,
                                  n_workgroups, st);
}

hipError_t launch_batched_apply(const BatchDev& b, int tensor, int precision, const PairConst& pc,
                                const void* pos, const void* frc, double* vel, int n_workgroups,
                                hipStream_t st)
{
    // APPLY reads positions as f64[3 total] (the caller stages them)
    return tensor == T_OSEEN
               ? launch_bt<T_OSEEN>(b, precision, SD_EULER, pc, (double*)pos, frc, vel, 0.0, -1,
                                    n_workgroups, st)
               : launch_bt<T_RPY>(b, precision, SD_EULER, pc, (double*)pos, frc, vel, 0.0, -1,
                                  n_workgroups, st);
}

// f32x4 / f64x4 positions -> f64[3 n]
__global__ void __launch_bounds__(256) k_unpack_f32(const float4* __restrict__ p,
                                                   double* __restrict__ x, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float4 v = p[i];
    x[3 * (size_t)i] = v.x;
    x[3 * (size_t)i + 1] = v.y;
    x[3 * (size_t)i + 2] = v.z;
}
__global__ void __launch_bounds__(256) k_unpack_f64(const double4* __restrict__ p,
                                                   double* __restrict__ x, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double4 v = p[i];
    x[3 * (size_t)i] = v.x;
    x[3 * (size_t)i + 1] = v.y;
    x[3 * (size_t)i + 2] = v.z;
}

// ---------------------------------------------------------------- the plan

struct GraphKey {
    double* x = nullptr;
    const void* frc = nullptr;
    double dt = 0.0;
    int64_t steps = -1;
    int32_t integ = -1, prec = -1, nwg = 0, wg = 0;
    bool operator==(const GraphKey& o) const
    {
        return x == o.x && frc == o.frc && dt == o.dt && steps == o.steps && integ == o.integ &&
               prec == o.prec && nwg == o.nwg && wg == o.wg;
    }
};

}  // namespace sd

struct sd_batch {
    int dev = 0;
    sd_params p{};
    int64_t n_clusters = 0;
    int64_t total = 0;
    int max_size = 0;
    int wg = 256;               // lanes per work-group (128, 256, 512)
    int per_cu = 0;             // resident work-groups per CU, 0 = automatic
    void* dmem = nullptr;       // offsets | order | counter
    int64_t* d_offsets = nullptr;
    int32_t* d_order = nullptr;
    int32_t* d_counter = nullptr;
    hipStream_t cap = nullptr;  // private stream used only for graph capture
    sd::GraphKey key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after the last replay
};

namespace sd {

static std::vector<sd_batch*> g_batches;  // live plans (for sd_release)
static std::mutex g_batches_mu;

// Waits for the last replay before the executable graph is destroyed.
static void drop_graph(sd_batch* b)
{
    if (b->exec && b->done) (void)hipEventSynchronize(b->done);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->key = GraphKey();
}

void batch_release_graphs()
{
    std::lock_guard<std::mutex> lk(g_batches_mu);
    for (sd_batch* b : g_batches) drop_graph(b);
}

// Persistent grid: per_cu work-groups per CU (automatic: 1024 lanes per CU,
// i.e. four waves per SIMD), limited by the 160 KiB of LDS per CU.
static int batch_workgroups(const sd_batch* b, int prec, int integ)
{
    const int cus = device_cus();
    const size_t lds = batched_lds_bytes(b->max_size, prec, integ, b->wg);
    const int want_cu = b->per_cu > 0 ? b->per_cu : 1024 / b->wg;
    int per_cu = (int)std::min<size_t>((size_t)want_cu,
                                       (160 * 1024) / std::max<size_t>(lds, 1));
    per_cu = std::max(per_cu, 1);
    const int64_t want = (int64_t)cus * per_cu;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, b->n_clusters));
}

static BatchDev batch_dev(const sd_batch* b)
{
    BatchDev d;
    d.offsets = b->d_offsets;
    d.order = b->d_order;
    d.counter = b->d_counter;
    d.n_clusters = (int)b->n_clusters;
    d.max_size = std::max(1, b->max_size);
    d.wg = b->wg;
    return d;
}

static sd_status check_batch(const sd_batch* b)
{
    if (!b) return fail(SD_EINVAL, "batch is NULL");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SD_EDEVICE, "hipGetDevice failed");
    if (dev != b->dev) return fail(SD_EINVAL, "batch plan belongs to device %d, current is %d",
                                   b->dev, dev);
    return SD_OK;
}

}  // namespace sd

using namespace sd;

extern "C" {

sd_status sd_batch_create(const sd_params* p, int64_t n_clusters, const int64_t* offsets,
                          sd_batch** out)
{
    sd_status st;
    if ((st = check_params(p)) || (st = check_free_space(p, "the batched path"))) return st;
    if (!out) return fail(SD_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_clusters < 1 || n_clusters > (int64_t(1) << 30))
        return fail(SD_EINVAL, "n_clusters must be in [1, 2^30]");
    if (!offsets) return fail(SD_EINVAL, "offsets is NULL");
    if (offsets[0] != 0) return fail(SD_EINVAL, "offsets[0] must be 0");
    int max_size = 0;
    for (int64_t c = 0; c < n_clusters; ++c) {
        const int64_t sz = offsets[c + 1] - offsets[c];
        if (sz < 0) return fail(SD_EINVAL, "offsets must be non-decreasing (cluster %lld)",
                                (long long)c);
        if (sz > SD_BATCH_MAX_CLUSTER)
            return fail(SD_EINVAL, "cluster %lld has %lld particles (max %d)", (long long)c,
                        (long long)sz, SD_BATCH_MAX_CLUSTER);
        max_size = std::max(max_size, (int)sz);
    }
    const int64_t total = offsets[n_clusters];
    if ((st = check_n(total))) return st;
    // longest first (stable, so equal sizes keep index order)
    std::vector<int32_t> order((size_t)n_clusters);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t bb) {
        return offsets[a + 1] - offsets[a] > offsets[bb + 1] - offsets[bb];
    });
    sd_batch* b = new sd_batch();
    b->p = *p;
    b->n_clusters = n_clusters;
    b->total = total;
    b->max_size = max_size;
    if (hipGetDevice(&b->dev) != hipSuccess) {
        delete b;
        return fail(SD_EDEVICE, "hipGetDevice failed");
    }
    const size_t ob = (size_t)(n_clusters + 1) * sizeof(int64_t);
    const size_t rb = (size_t)n_clusters * sizeof(int32_t);
    if (hipMalloc(&b->dmem, ob + rb + 256) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return fail(SD_ENOMEM, "plan allocation failed");
    }
    b->d_offsets = (int64_t*)b->dmem;
    b->d_order = (int32_t*)((char*)b->dmem + ob);
    b->d_counter = (int32_t*)((char*)b->dmem + ((ob + rb + 63) & ~(size_t)63));
    if (hipMemcpy(b->d_offsets, offsets, ob, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_order, order.data(), rb, hipMemcpyHostToDevice) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        if (b->cap) (void)hipStreamDestroy(b->cap);
        (void)hipFree(b->dmem);
        delete b;
        return fail(SD_EDEVICE, "plan upload failed");
    }
    {
        std::lock_guard<std::mutex> lk(g_batches_mu);
        g_batches.push_back(b);
    }
    *out = b;
    return SD_OK;
}

sd_status sd_batch_destroy(sd_batch* b)
{
    if (!b) return SD_OK;
    {   // off the list first, so that sd_release no longer reaches it
        std::lock_guard<std::mutex> lk(g_batches_mu);
        g_batches.erase(std::remove(g_batches.begin(), g_batches.end(), b), g_batches.end());
    }
    (void)hipDeviceSynchronize();
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->dmem) (void)hipFree(b->dmem);
    delete b;
    return SD_OK;
}

int64_t sd_batch_particles(const sd_batch* b)
{
    return b ? b->total : -1;
}

sd_status mobility_apply_batched(sd_batch* b, const void* pos, const void* force, double* vel,
                                 int32_t precision, void* stream)
{
    sd_status st;
    if ((st = check_batch(b)) || (st = check_precision(precision))) return st;
    const size_t al = vec4_align(precision);
    if ((st = check_ptr(pos, al, "pos")) || (st = check_ptr(force, al, "force")) ||
        (st = check_ptr(vel, 8, "vel")))
        return st;
    hipStream_t hs = (hipStream_t)stream;
    void* x64 = nullptr;
    if ((st = ws_get(WS_STAGE, 3 * (size_t)b->total * sizeof(double), &x64))) return st;
    const int n = (int)b->total;
    if (precision == SD_FP64)
        hipLaunchKernelGGL(k_unpack_f64, dim3((n + 255) / 256), dim3(256), 0, hs,
                           (const double4*)pos, (double*)x64, n);
    else
        hipLaunchKernelGGL(k_unpack_f32, dim3((n + 255) / 256), dim3(256), 0, hs,
                           (const float4*)pos, (double*)x64, n);
    const int nwg = batch_workgroups(b, precision, SD_EULER);
    hipError_t e = launch_fill_i32(b->d_counter, 0, 1, hs);
    if (e == hipSuccess)
        e = launch_batched_apply(batch_dev(b), b->p.tensor, precision, pair_const(&b->p), x64,
                                 force, vel, nwg, hs);
    if (e != hipSuccess) return fail(SD_EDEVICE, "batched launch: %s", hipGetErrorString(e));
    return SD_OK;
}

sd_status sd_run_batched(sd_batch* b, double* x, const void* force, double dt, int64_t steps,
                         int32_t integrator, int32_t precision, int32_t use_graph, void* stream)
{
    sd_status st;
    if ((st = check_batch(b)) || (st = check_precision(precision))) return st;
    if ((st = check_ptr(x, 8, "x")) || (st = check_ptr(force, vec4_align(precision), "force")))
        return st;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SD_EINVAL, "dt must be finite and > 0");
    if (steps < 0 || steps > INT32_MAX) return fail(SD_EINVAL, "steps must be in [0, 2^31)");
    if (integrator != SD_EULER && integrator != SD_AB2) return fail(SD_EINVAL, "unknown integrator");
    if (steps == 0) return SD_OK;
    hipStream_t hs = (hipStream_t)stream;
    const int nwg = batch_workgroups(b, precision, integrator);
    const PairConst pc = pair_const(&b->p);
    const BatchDev d = batch_dev(b);
    if (!use_graph) {
        hipError_t e = launch_fill_i32(b->d_counter, 0, 1, hs);
        if (e == hipSuccess)
            e = launch_batched_run(d, b->p.tensor, precision, pc, x, force, dt, (int)steps,
                                   integrator, nwg, hs);
        if (e != hipSuccess) return fail(SD_EDEVICE, "batched launch: %s", hipGetErrorString(e));
        return SD_OK;
    }
    GraphKey key;
    key.x = x;
    key.frc = force;
    key.dt = dt;
    key.steps = steps;
    key.integ = integrator;
    key.prec = precision;
    key.nwg = nwg;
    key.wg = b->wg;
    if (!b->exec || !(b->key == key)) {
        drop_graph(b);
        // capture [queue reset (fill kernel, no memset node), persistent kernel]
        if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(SD_EDEVICE, "hipStreamBeginCapture failed");
        hipError_t e = launch_fill_i32(b->d_counter, 0, 1, b->cap);
        if (e == hipSuccess)
            e = launch_batched_run(d, b->p.tensor, precision, pc, x, force, dt, (int)steps,
                                   integrator, nwg, b->cap);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap, &g);
        if (e != hipSuccess || e2 != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return fail(SD_EDEVICE, "graph capture failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        hipGraphExec_t ex = nullptr;
        if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(SD_EDEVICE, "hipGraphInstantiate failed");
        }
        b->graph = g;
        b->exec = ex;
        b->key = key;
    }
    if (hipGraphLaunch(b->exec, hs) != hipSuccess) return fail(SD_EDEVICE, "hipGraphLaunch failed");
    if (hipEventRecord(b->done, hs) != hipSuccess) return fail(SD_EDEVICE, "event record failed");
    return SD_OK;
}

sd_status sd_batch_set_config(sd_batch* b, int32_t workgroup, int32_t per_cu)
{
    sd_status st;
    if ((st = check_batch(b))) return st;
    if (workgroup == 0) workgroup = 256;
    if (workgroup != 128 && workgroup != 256 && workgroup != 512)
        return fail(SD_EINVAL, "workgroup must be 128, 256 or 512 (got %d)", workgroup);
    if (per_cu < 0 || per_cu > 16) return fail(SD_EINVAL, "per_cu must be in [0, 16]");
    if (b->wg != workgroup || b->per_cu != per_cu) drop_graph(b);
    b->wg = workgroup;
    b->per_cu = per_cu;
    return SD_OK;
}

sd_status sd_batch_get_config(const sd_batch* b, int32_t* workgroup, int32_t* per_cu)
{
    sd_status st;
    if ((st = check_batch(b))) return st;
    if (!workgroup || !per_cu) return fail(SD_EINVAL, "output pointer is NULL");
    *workgroup = b->wg;
    *per_cu = b->per_cu;
    return SD_OK;
}

sd_status sd_batch_autotune(sd_batch* b, const double* x, const void* force, double dt,
                            int64_t steps, int32_t integrator, int32_t precision, char* report,
                            int64_t report_len, void* stream)
{
    sd_status st;
    if ((st = check_batch(b)) || (st = check_precision(precision))) return st;
    if ((st = check_ptr(x, 8, "x")) || (st = check_ptr(force, vec4_align(precision), "force")))
        return st;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SD_EINVAL, "dt must be finite and > 0");
    if (steps < 1 || steps > INT32_MAX) return fail(SD_EINVAL, "steps must be in [1, 2^31)");
    if (integrator != SD_EULER && integrator != SD_AB2) return fail(SD_EINVAL, "unknown integrator");
    hipStream_t hs = (hipStream_t)stream;
    const size_t bytes = 3 * (size_t)b->total * sizeof(double);
    void* scratch = nullptr;
    if ((st = ws_get(WS_TUNE, bytes, &scratch))) return st;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(SD_EDEVICE, "hipEventCreate failed");
    const int wg0 = b->wg, pc0 = b->per_cu;
    struct Res {
        int wg, per_cu;
        float ms;
    };
    std::vector<Res> res;
    const PairConst pc = pair_const(&b->p);
    // every candidate runs the caller's steps on a copy of x (x is not changed):
    // one warm-up, then the median of three timed launches
    for (int wg : { 128, 256, 512 })
        for (int pcu : { 0, 1, 2 }) {
            const int per_cu = pcu == 0 ? 0 : (pcu == 1 ? 512 / wg : 2048 / wg);
            if (per_cu > 16) continue;
            b->wg = wg;
            b->per_cu = per_cu;
            const int nwg = batch_workgroups(b, precision, integrator);
            const BatchDev d = batch_dev(b);
            float t[4] = { 0.f, 0.f, 0.f, 0.f };
            for (int r = 0; r < 4 && !st; ++r) {
                hipError_t e = hipMemcpyAsync(scratch, x, bytes, hipMemcpyDeviceToDevice, hs);
                if (e == hipSuccess) e = launch_fill_i32(b->d_counter, 0, 1, hs);
                if (e == hipSuccess) e = hipEventRecord(e0, hs);
                if (e == hipSuccess)
                    e = launch_batched_run(d, b->p.tensor, precision, pc, (double*)scratch, force,
                                           dt, (int)steps, integrator, nwg, hs);
                if (e == hipSuccess) e = hipEventRecord(e1, hs);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&t[r], e0, e1);
                if (e != hipSuccess) st = fail(SD_EDEVICE, "batched autotune: %s",
                                               hipGetErrorString(e));
            }
            if (st) break;
            std::sort(t + 1, t + 4);
            res.push_back({ wg, per_cu, t[2] });
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->wg = wg0;
    b->per_cu = pc0;
    if (st) return st;
    std::sort(res.begin(), res.end(), [](const Res& a, const Res& c) { return a.ms < c.ms; });
    drop_graph(b);
    b->wg = res[0].wg;
    b->per_cu = res[0].per_cu;
    if (report && report_len > 0) {
        std::string js = "{\"best\": {\"workgroup\": " + std::to_string(res[0].wg) +
                         ", \"per_cu\": " + std::to_string(res[0].per_cu) +
                         ", \"ms\": " + std::to_string(res[0].ms) + "}, \"candidates\": [";
        for (size_t k = 0; k < res.size(); ++k)
            js += (k ? ", " : "") + std::string("{\"workgroup\": ") + std::to_string(res[k].wg) +
                  ", \"per_cu\": " + std::to_string(res[k].per_cu) +
                  ", \"ms\": " + std::to_string(res[k].ms) + "}";
        js += "]}";
        std::snprintf(report, (size_t)report_len, "%s", js.c_str());
    }
    return SD_OK;
}

}  // extern "C"
