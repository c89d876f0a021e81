// cluster_run.hip -- the numerical-stability study of Sec. 4: long Euler runs
// of one small free-space cluster (the four sedimenting spheres of Fig. 4)
// with the precision of (a) the accumulation of the hydrodynamic interactions
// and (b) the positions chosen per run.
//
// A run is latency-bound (n <= 64 spheres, tens of millions of dependent
// steps), so each run is one wave that keeps its cluster in registers and LDS
// for every step of a call: lane i owns sphere i, the wave publishes the
// positions in LDS, every lane sums over j in the same order 0..n-1, and the
// Euler update happens in the lane.  Independent runs (precision variants,
// time steps) are independent work-groups of the same launch.
#include "pair_terms.h"
#include "sd.h"
#include "sd_host.h"
#include "sd_internal.h"

#include <cmath>
#include <vector>

namespace sd {

struct ClusterRunDev {
    int acc, pos;
    double dt;
    long long steps, stride;
    long long frame0;   // index of the run's first frame in traj
};

// Error-free FP32 sum: a + b = s + e exactly (Knuth's two-sum).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Double-single (hi, lo) += (bh, bl), renormalised so that |lo| <= ulp(hi)/2.
__device__ __forceinline__ void ds_add(float& hi, float& lo, float bh, float bl)
{
    float s, e;
    two_sum(hi, bh, s, e);
    e += lo + bl;
    hi = s + e;
    lo = e - (hi - s);
}

// One run, its precisions fixed at compile time (ACC: sd_acc_mode, POS:
// sd_pos_mode), so that the step loop carries no mode branches.
template <int TENSOR, int ACC, int POS>
__device__ __forceinline__ void cluster_body(const ClusterRunDev& R, int n, const PairConst& pc,
                                             double* __restrict__ state,
                                             const double* __restrict__ force,
                                             double* __restrict__ traj, float (*s_hi)[64],
                                             float (*s_lo)[64], double (*s_x)[64],
                                             double (*s_f)[64])
{
    const int i = threadIdx.x;
    const bool act = i < n;
    double* st = state + (size_t)blockIdx.x * 6 * (size_t)n;

    // the run's position representation: FP32 (xl = 0), double-single (xh, xl)
    // or FP64 (x64; xh, xl its FP32 head and tail for the FP32 differences)
    float xh[3], xl[3];
    double x64[3], f[3];
    for (int k = 0; k < 3; ++k) {
        const double v = act ? st[3 * i + k] + st[3 * (size_t)n + 3 * i + k] : 0.0;
        f[k] = act ? force[3 * i + k] : 0.0;
        xh[k] = (float)v;
        xl[k] = (POS == SD_POS_FP32) ? 0.0f : (float)(v - (double)xh[k]);
        x64[k] = (POS == SD_POS_FP64) ? v : (double)xh[k] + (double)xl[k];
    }
    const float gamma = pc.gamma_f, m3g = pc.m3gamma_f, thr2 = pc.thr2_f;
    // the constant forces stay in LDS for the whole call
    for (int k = 0; k < 3; ++k) s_f[k][i] = f[k];

    long long frame = R.frame0, since = 0;  // next frame, steps since the last one
    for (long long step = 0; step < R.steps; ++step) {
        for (int k = 0; k < 3; ++k) {
            if (ACC != SD_ACC_FP64) s_hi[k][i] = xh[k];
            if (ACC != SD_ACC_FP64 && POS != SD_POS_FP32) s_lo[k][i] = xl[k];
            s_x[k][i] = x64[k];
        }
        __syncthreads();
        double v[3];
        if (ACC == SD_ACC_FP64) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                near_term<TENSOR>(pc, x64[0] - s_x[0][j], x64[1] - s_x[1][j], x64[2] - s_x[2][j],
                                  s_f[0][j], s_f[1][j], s_f[2][j], a0, a1, a2);
            }
            v[0] = pc.mu0 * f[0] + a0;
            v[1] = pc.mu0 * f[1] + a1;
            v[2] = pc.mu0 * f[2] + a2;
        } else {
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;  // sums (scaled units, Eq. 7 / alpha)
            float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;  // Kahan compensation or double-single tail
            double n0 = 0.0, n1 = 0.0, n2 = 0.0;    // FP64 near pairs (physical units)
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                float dx = xh[0] - s_hi[0][j], dy = xh[1] - s_hi[1][j], dz = xh[2] - s_hi[2][j];
                if (POS != SD_POS_FP32) {
                    dx += xl[0] - s_lo[0][j];
                    dy += xl[1] - s_lo[1][j];
                    dz += xl[2] - s_lo[2][j];
                }
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float fx = (float)s_f[0][j], fy = (float)s_f[1][j], fz = (float)s_f[2][j];
                if (r2 < thr2) {
                    near_term<TENSOR>(pc, x64[0] - s_x[0][j], x64[1] - s_x[1][j],
                                      x64[2] - s_x[2][j], (double)fx, (double)fy, (double)fz, n0,
                                      n1, n2);
                    continue;
                }
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float rinv2 = rinv * rinv, rinv3 = rinv2 * rinv;
                float A, Bt;
                if (TENSOR == T_OSEEN) {
                    A = rinv;
                    Bt = rinv3;
                } else {
                    A = fmaf(gamma, rinv3, rinv);
                    Bt = rinv3 * fmaf(m3g, rinv2, 1.0f);
                }
                const float sB = Bt * fmaf(dx, fx, fmaf(dy, fy, dz * fz));
                const float t0 = fmaf(A, fx, sB * dx);
                const float t1 = fmaf(A, fy, sB * dy);
                const float t2 = fmaf(A, fz, sB * dz);
                if (ACC == SD_ACC_FP32) {
                    s0 += t0;
                    s1 += t1;
                    s2 += t2;
                } else if (ACC == SD_ACC_KAHAN) {
                    const float y0 = t0 - c0, y1 = t1 - c1, y2 = t2 - c2;
                    const float u0 = s0 + y0, u1 = s1 + y1, u2 = s2 + y2;
                    c0 = (u0 - s0) - y0;
                    c1 = (u1 - s1) - y1;
                    c2 = (u2 - s2) - y2;
                    s0 = u0;
                    s1 = u1;
                    s2 = u2;
                } else {
                    ds_add(s0, c0, t0, 0.0f);
                    ds_add(s1, c1, t1, 0.0f);
                    ds_add(s2, c2, t2, 0.0f);
                }
            }
            // Kahan: the sum is s - c; double-single: s + c
            const double sg = (ACC == SD_ACC_KAHAN) ? -1.0 : 1.0;
            v[0] = pc.mu0 * f[0] + pc.alpha * ((double)s0 + sg * (double)c0) + n0;
            v[1] = pc.mu0 * f[1] + pc.alpha * ((double)s1 + sg * (double)c1) + n1;
            v[2] = pc.mu0 * f[2] + pc.alpha * ((double)s2 + sg * (double)c2) + n2;
        }
        // Euler update in the run's position precision
        for (int k = 0; k < 3; ++k) {
            const double inc = R.dt * v[k];
            if (POS == SD_POS_FP32) {
                xh[k] = xh[k] + (float)inc;
                x64[k] = (double)xh[k];
            } else if (POS == SD_POS_DS) {
                const float ih = (float)inc;
                ds_add(xh[k], xl[k], ih, (float)(inc - (double)ih));
                x64[k] = (double)xh[k] + (double)xl[k];
            } else {
                x64[k] += inc;
                xh[k] = (float)x64[k];
                xl[k] = (float)(x64[k] - (double)xh[k]);
            }
        }
        if (R.stride > 0 && ++since == R.stride) {
            since = 0;
            if (act) {
                double* fr = traj + (size_t)frame * 3 * (size_t)n;
                fr[3 * i] = x64[0];
                fr[3 * i + 1] = x64[1];
                fr[3 * i + 2] = x64[2];
            }
            ++frame;
        }
        __syncthreads();  // every lane has read the positions before they change
    }
    if (act)
        for (int k = 0; k < 3; ++k) {
            if (POS == SD_POS_DS) {
                st[3 * i + k] = (double)xh[k];
                st[3 * (size_t)n + 3 * i + k] = (double)xl[k];
            } else {
                st[3 * i + k] = (POS == SD_POS_FP32) ? (double)xh[k] : x64[k];
                st[3 * (size_t)n + 3 * i + k] = 0.0;
            }
        }
}


template <int TENSOR>
__global__ void __launch_bounds__(64)
k_cluster_run(const ClusterRunDev* __restrict__ runs, int n, PairConst pc,
              double* __restrict__ state, const double* __restrict__ force,
              double* __restrict__ traj)
{
    __shared__ float s_hi[3][64], s_lo[3][64];
    __shared__ double s_x[3][64], s_f[3][64];
    const ClusterRunDev R = runs[blockIdx.x];
#define SD_CR(A, P)                                                                            \
    if (R.acc == A && R.pos == P) {                                                            \
        cluster_body<TENSOR, A, P>(R, n, pc, state, force, traj, s_hi, s_lo, s_x, s_f);        \
        return;                                                                                \
    }
    SD_CR(0, 0) SD_CR(0, 1) SD_CR(0, 2) SD_CR(1, 0) SD_CR(1, 1) SD_CR(1, 2)
    SD_CR(2, 0) SD_CR(2, 1) SD_CR(2, 2) SD_CR(3, 0) SD_CR(3, 1) SD_CR(3, 2)
#undef SD_CR
}

}  // namespace sd

using namespace sd;

extern "C" sd_status sd_cluster_run(const sd_params* p, int64_t n, int32_t runs,
                                    const sd_cluster_spec* specs, double* state,
                                    const double* force, double* traj, void* stream)
{
    sd_status st;
    if ((st = check_params(p)) || (st = check_free_space(p, "sd_cluster_run"))) return st;
    if (n < 1 || n > SD_CLUSTER_MAX_N)
        return fail(SD_EINVAL, "n must be in [1, %d] (got %lld)", SD_CLUSTER_MAX_N, (long long)n);
    if (runs < 1 || runs > SD_CLUSTER_MAX_RUNS)
        return fail(SD_EINVAL, "runs must be in [1, %d]", SD_CLUSTER_MAX_RUNS);
    if (!specs) return fail(SD_EINVAL, "specs is NULL");
    if ((st = check_ptr(state, 8, "state")) || (st = check_ptr(force, 8, "force"))) return st;
    std::vector<ClusterRunDev> rec((size_t)runs);
    long long frames = 0;
    for (int r = 0; r < runs; ++r) {
        const sd_cluster_spec& s = specs[r];
        if (s.acc < SD_ACC_FP32 || s.acc > SD_ACC_FP64)
            return fail(SD_EINVAL, "run %d: unknown accumulation mode %d", r, s.acc);
        if (s.pos < SD_POS_FP32 || s.pos > SD_POS_FP64)
            return fail(SD_EINVAL, "run %d: unknown position mode %d", r, s.pos);
        if (!(s.dt > 0.0) || !std::isfinite(s.dt))
            return fail(SD_EINVAL, "run %d: dt must be finite and > 0", r);
        if (s.steps < 0 || s.stride < 0)
            return fail(SD_EINVAL, "run %d: steps and stride must be >= 0", r);
        rec[r].acc = s.acc;
        rec[r].pos = s.pos;
        rec[r].dt = s.dt;
        rec[r].steps = s.steps;
        rec[r].stride = s.stride;
        rec[r].frame0 = frames;
        if (s.stride > 0) frames += s.steps / s.stride;
    }
    if (frames > 0 && (st = check_ptr(traj, 8, "traj"))) return st;
    hipStream_t hs = (hipStream_t)stream;
    void* buf = nullptr;
    if ((st = ws_get(WS_CLUSTER, rec.size() * sizeof(ClusterRunDev), &buf))) return st;
    // the run records go through library workspace; the upload is complete
    // (and the host vector free to go) when the call returns
    if (hipMemcpyAsync(buf, rec.data(), rec.size() * sizeof(ClusterRunDev),
                       hipMemcpyHostToDevice, hs) != hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess)
        return fail(SD_EDEVICE, "cluster-run record upload failed");
    const PairConst pc = pair_const(p);
    if (p->tensor == SD_OSEEN)
        hipLaunchKernelGGL((k_cluster_run<T_OSEEN>), dim3(runs), dim3(64), 0, hs,
                           (const ClusterRunDev*)buf, (int)n, pc, state, force, traj);
    else
        hipLaunchKernelGGL((k_cluster_run<T_RPY>), dim3(runs), dim3(64), 0, hs,
                           (const ClusterRunDev*)buf, (int)n, pc, state, force, traj);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SD_EDEVICE, "cluster-run launch: %s", hipGetErrorString(e));
    return SD_OK;
}
