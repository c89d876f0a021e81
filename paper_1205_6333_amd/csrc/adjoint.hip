// adjoint.hip -- reverse mode of the mobility product and of the Euler time
// loop.
//
// For a cotangent lam (dL/dv) the position gradient of lam . M(x) F is
//   g_i = sum_{j != i} grad_r [ lam_i . T(r) F_j + lam_j . T(r) F_i ],  r = x_i - x_j
// (x_i enters v_i through T(x_i - x_j) and v_j through T(x_j - x_i); T is even
// in r, so both terms are taken at r = x_i - x_j with a plus sign).  Writing
// T = alpha [A'(r) I + Bt'(r) r r]:
//   grad_r [u.T.w] = alpha [ (dA'/dr (u.w) + dBt'/dr (u.r)(w.r)) rhat
//                            + Bt' ((w.r) u + (u.r) w) ].
// The force gradient is M(x)^T lam = M(x) lam (block symmetry of the mobility
// matrix): mu0 lam_i + sum_{j != i} T(r) lam_j.  The adjoint pair kernel
// accumulates it in the same pass (lam_j . d is needed for the position
// gradient anyway), so one kernel gives both gradients.
#include "sd.h"
#include "sd_host.h"
#include "sd_internal.h"

#include <algorithm>
#include <cmath>

namespace sd {

#define SD_FAR_I (-1.0e15f)
#define SD_FAR_J (1.0e15f)

// FP64 gradient contribution of one near pair (d = x_i - x_j, r^2 below threshold).
template <int TENSOR>
__device__ __forceinline__ void adj_near(const PairConst& pc, double d0, double d1, double d2,
                                         const double* li, const double* fj, const double* lj,
                                         const double* fi, double& n0, double& n1, double& n2)
{
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (r2 == 0.0) return;  // coincident spheres: no gradient (measure-zero set)
    const double r = sqrt(r2);
    double Bt, dA, dBt;     // T = A I + Bt d d (physical units); derivatives in r
    if (TENSOR == T_OSEEN) {
        Bt = pc.alpha / (r2 * r);
        dA = -pc.alpha / r2;
        dBt = -3.0 * pc.alpha / (r2 * r2);
    } else if (pc.overlap && r < 2.0 * pc.a) {
        Bt = pc.mu0 * 3.0 / (32.0 * pc.a * r);
        dA = -pc.mu0 * 9.0 / (32.0 * pc.a);
        dBt = -pc.mu0 * 3.0 / (32.0 * pc.a * r2);
    } else {
        const double ri = 1.0 / r, ri2 = ri * ri, ri3 = ri * ri2, ri4 = ri2 * ri2;
        Bt = pc.alpha * (ri3 - 3.0 * pc.gamma * ri3 * ri2);
        dA = pc.alpha * (-ri2 - 3.0 * pc.gamma * ri4);
        dBt = pc.alpha * (-3.0 * ri4 + 15.0 * pc.gamma * ri4 * ri2);
    }
    const double d[3] = { d0, d1, d2 };
    double uw = 0.0, li_d = 0.0, fj_d = 0.0, lj_d = 0.0, fi_d = 0.0;
    for (int k = 0; k < 3; ++k) {
        uw += li[k] * fj[k] + lj[k] * fi[k];
        li_d += li[k] * d[k];
        fj_d += fj[k] * d[k];
        lj_d += lj[k] * d[k];
        fi_d += fi[k] * d[k];
    }
    const double c1 = (dA * uw + dBt * (li_d * fj_d + lj_d * fi_d)) / r;
    double g[3];
    for (int k = 0; k < 3; ++k)
        g[k] = c1 * d[k] + Bt * (fj_d * li[k] + li_d * fj[k] + fi_d * lj[k] + lj_d * fi[k]);
    n0 += g[0];
    n1 += g[1];
    n2 += g[2];
}

struct LaneAdj {
    float x, y, z;       // position of i
    float lx, ly, lz;    // cotangent lam_i
    float fx, fy, fz;    // force F_i
    float s0, s1, s2, c0, c1, c2;        // position gradient (Kahan)
    float g0, g1, g2, e0, e1, e2;        // (M lam)_i pair part (Kahan)
    double n0, n1, n2;                   // near pairs, position gradient
    double m0, m1, m2;                   // near pairs, M lam
    int i;
};

// FP64 T(r) lam_j of one near pair (d = x_i - x_j), the same definitions as
// the product kernels.
template <int TENSOR>
__device__ __forceinline__ void adj_near_mlam(const PairConst& pc, double d0, double d1, double d2,
                                              const double* lj, double& m0, double& m1,
                                              double& m2)
{
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (r2 == 0.0) {
        if (TENSOR == T_RPY && pc.overlap) {
            m0 += pc.mu0 * lj[0];
            m1 += pc.mu0 * lj[1];
            m2 += pc.mu0 * lj[2];
        }
        return;
    }
    const double r = sqrt(r2);
    double cI, cD;
    if (TENSOR == T_OSEEN) {
        cI = pc.alpha / r;
        cD = cI / r2;
    } else if (pc.overlap && r < 2.0 * pc.a) {
        cI = pc.mu0 * (1.0 - 9.0 * r / (32.0 * pc.a));
        cD = pc.mu0 * 3.0 / (32.0 * pc.a * r);
    } else {
        const double ri = 1.0 / r, ri2 = ri * ri, ri3 = ri * ri2;
        cI = pc.alpha * (ri + pc.gamma * ri3);
        cD = pc.alpha * ri3 * (1.0 - 3.0 * pc.gamma * ri2);
    }
    const double dl = d0 * lj[0] + d1 * lj[1] + d2 * lj[2];
    m0 += cI * lj[0] + cD * dl * d0;
    m1 += cI * lj[1] + cD * dl * d1;
    m2 += cI * lj[2] + cD * dl * d2;
}

// masked pair (handles near pairs and the self pair in FP64)
template <int TENSOR>
__device__ __forceinline__ void adj_pair_masked(LaneAdj& L, const float4 pj, const float4 fj,
                                                const float4 lj, int jg, int n,
                                                const PairConst& pc, float gamma,
                                                const double* __restrict__ x64)
{
    const float dx = L.x - pj.x, dy = L.y - pj.y, dz = L.z - pj.z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const bool nr = r2 < pc.thr2_f;
    if (nr) {
        if (jg != L.i && L.i < n && jg < n) {
            double d0, d1, d2;
            if (x64) {
                d0 = x64[3 * (size_t)L.i] - x64[3 * (size_t)jg];
                d1 = x64[3 * (size_t)L.i + 1] - x64[3 * (size_t)jg + 1];
                d2 = x64[3 * (size_t)L.i + 2] - x64[3 * (size_t)jg + 2];
            } else {
                d0 = (double)L.x - (double)pj.x;
                d1 = (double)L.y - (double)pj.y;
                d2 = (double)L.z - (double)pj.z;
            }
            const double li[3] = { L.lx, L.ly, L.lz }, fi[3] = { L.fx, L.fy, L.fz };
            const double fjd[3] = { fj.x, fj.y, fj.z }, ljd[3] = { lj.x, lj.y, lj.z };
            adj_near<TENSOR>(pc, d0, d1, d2, li, fjd, ljd, fi, L.n0, L.n1, L.n2);
            adj_near_mlam<TENSOR>(pc, d0, d1, d2, ljd, L.m0, L.m1, L.m2);
        }
        return;
    }
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rinv2 = rinv * rinv, rinv3 = rinv2 * rinv, rinv5 = rinv3 * rinv2;
    float Bt, P, Q;
    if (TENSOR == T_OSEEN) {
        Bt = rinv3;
        P = -rinv3;
        Q = -3.0f * rinv5;
    } else {
        Bt = fmaf(-3.0f * gamma, rinv5, rinv3);
        P = -fmaf(3.0f * gamma, rinv5, rinv3);
        Q = rinv5 * fmaf(15.0f * gamma, rinv2, -3.0f);
    }
    const float li_fj = fmaf(L.lx, fj.x, fmaf(L.ly, fj.y, L.lz * fj.z));
    const float lj_fi = fmaf(lj.x, L.fx, fmaf(lj.y, L.fy, lj.z * L.fz));
    const float li_d = fmaf(L.lx, dx, fmaf(L.ly, dy, L.lz * dz));
    const float fj_d = fmaf(fj.x, dx, fmaf(fj.y, dy, fj.z * dz));
    const float lj_d = fmaf(lj.x, dx, fmaf(lj.y, dy, lj.z * dz));
    const float fi_d = fmaf(L.fx, dx, fmaf(L.fy, dy, L.fz * dz));
    const float q = fmaf(li_d, fj_d, lj_d * fi_d);
    const float c1 = fmaf(P, li_fj + lj_fi, Q * q);
    const float w0 = fmaf(fj_d, L.lx, fmaf(li_d, fj.x, fmaf(fi_d, lj.x, lj_d * L.fx)));
    const float w1 = fmaf(fj_d, L.ly, fmaf(li_d, fj.y, fmaf(fi_d, lj.y, lj_d * L.fy)));
    const float w2 = fmaf(fj_d, L.lz, fmaf(li_d, fj.z, fmaf(fi_d, lj.z, lj_d * L.fz)));
    const float y0 = fmaf(c1, dx, fmaf(Bt, w0, -L.c0));
    const float y1 = fmaf(c1, dy, fmaf(Bt, w1, -L.c1));
    const float y2 = fmaf(c1, dz, fmaf(Bt, w2, -L.c2));
    const float t0 = L.s0 + y0, t1 = L.s1 + y1, t2 = L.s2 + y2;
    L.c0 = (t0 - L.s0) - y0;
    L.c1 = (t1 - L.s1) - y1;
    L.c2 = (t2 - L.s2) - y2;
    L.s0 = t0;
    L.s1 = t1;
    L.s2 = t2;
    // M lam: A lam_j + Bt (d . lam_j) d
    const float A = (TENSOR == T_OSEEN) ? rinv : fmaf(gamma, rinv3, rinv);
    const float sl = Bt * lj_d;
    const float z0 = fmaf(A, lj.x, fmaf(sl, dx, -L.e0));
    const float z1 = fmaf(A, lj.y, fmaf(sl, dy, -L.e1));
    const float z2 = fmaf(A, lj.z, fmaf(sl, dz, -L.e2));
    const float u0 = L.g0 + z0, u1 = L.g1 + z1, u2 = L.g2 + z2;
    L.e0 = (u0 - L.g0) - z0;
    L.e1 = (u1 - L.g1) - z1;
    L.e2 = (u2 - L.g2) - z2;
    L.g0 = u0;
    L.g1 = u1;
    L.g2 = u2;
}

// LDS-tiled adjoint pair kernel: tiles of BLOCK j-particles (position, force,
// cotangent: 48 B each); groups of 4 j with one near test per group, Kahan
// compensation once per group on the fast path.
template <int TENSOR, int BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_adjoint_f32(const float4* __restrict__ pos, const float4* __restrict__ frc,
              const float4* __restrict__ lam, const double* __restrict__ x64, int n, int jchunk,
              PairConst pc, double* __restrict__ partial, double* __restrict__ partial_f)
{
    __shared__ float4 s_pos[BLOCK];
    __shared__ float4 s_frc[BLOCK];
    __shared__ float4 s_lam[BLOCK];
    const int tid = threadIdx.x;
    const int s = blockIdx.y;
    LaneAdj L;
    L.i = blockIdx.x * BLOCK + tid;
    {
        float4 p = make_float4(SD_FAR_I, SD_FAR_I, SD_FAR_I, 0.0f), f = make_float4(0, 0, 0, 0),
               l = make_float4(0, 0, 0, 0);
        if (L.i < n) {
            p = pos[L.i];
            f = frc[L.i];
            l = lam[L.i];
        }
        L.x = p.x; L.y = p.y; L.z = p.z;
        L.fx = f.x; L.fy = f.y; L.fz = f.z;
        L.lx = l.x; L.ly = l.y; L.lz = l.z;
        L.s0 = L.s1 = L.s2 = L.c0 = L.c1 = L.c2 = 0.0f;
        L.g0 = L.g1 = L.g2 = L.e0 = L.e1 = L.e2 = 0.0f;
        L.n0 = L.n1 = L.n2 = 0.0;
        L.m0 = L.m1 = L.m2 = 0.0;
    }
    const float gamma = pc.gamma_f, thr2 = pc.thr2_f;
    const float g3 = -3.0f * gamma, m3g = 3.0f * gamma, g15 = 15.0f * gamma;
    const int jbeg = s * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const float4 far_j = make_float4(SD_FAR_J, SD_FAR_J, SD_FAR_J, 0.0f);
    const float4 zero4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 rp = far_j, rf = zero4, rl = zero4;
    if (jbeg + tid < jend) {
        rp = pos[jbeg + tid];
        rf = frc[jbeg + tid];
        rl = lam[jbeg + tid];
    }
    for (int jt = jbeg; jt < jend; jt += BLOCK) {
        __syncthreads();
        s_pos[tid] = rp;
        s_frc[tid] = rf;
        s_lam[tid] = rl;
        __syncthreads();
        const int jn = jt + BLOCK + tid;
        rp = far_j;
        rf = zero4;
        rl = zero4;
        if (jn < jend) {
            rp = pos[jn];
            rf = frc[jn];
            rl = lam[jn];
        }
        for (int k = 0; k < BLOCK; k += 4) {
            float4 pj[4], fj[4], lj[4];
            float dx[4], dy[4], dz[4], r2[4];
            float rmin = 3.0e38f;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                pj[u] = s_pos[k + u];
                fj[u] = s_frc[k + u];
                lj[u] = s_lam[k + u];
                dx[u] = L.x - pj[u].x;
                dy[u] = L.y - pj[u].y;
                dz[u] = L.z - pj[u].z;
                r2[u] = fmaf(dx[u], dx[u], fmaf(dy[u], dy[u], dz[u] * dz[u]));
                rmin = fminf(rmin, r2[u]);
            }
            if (__builtin_amdgcn_ballot_w64(rmin < thr2) != 0) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    adj_pair_masked<TENSOR>(L, pj[u], fj[u], lj[u], jt + k + u, n, pc, gamma, x64);
                continue;
            }
            float y0 = -L.c0, y1 = -L.c1, y2 = -L.c2;
            float z0 = -L.e0, z1 = -L.e1, z2 = -L.e2;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float rinv = __builtin_amdgcn_rsqf(r2[u]);
                const float rinv2 = rinv * rinv, rinv3 = rinv2 * rinv, rinv5 = rinv3 * rinv2;
                float Bt, P, Q;
                if (TENSOR == T_OSEEN) {
                    Bt = rinv3;
                    P = -rinv3;
                    Q = -3.0f * rinv5;
                } else {
                    Bt = fmaf(g3, rinv5, rinv3);
                    P = -fmaf(m3g, rinv5, rinv3);
                    Q = rinv5 * fmaf(g15, rinv2, -3.0f);
                }
                const float li_fj = fmaf(L.lx, fj[u].x, fmaf(L.ly, fj[u].y, L.lz * fj[u].z));
                const float lj_fi = fmaf(lj[u].x, L.fx, fmaf(lj[u].y, L.fy, lj[u].z * L.fz));
                const float li_d = fmaf(L.lx, dx[u], fmaf(L.ly, dy[u], L.lz * dz[u]));
                const float fj_d = fmaf(fj[u].x, dx[u], fmaf(fj[u].y, dy[u], fj[u].z * dz[u]));
                const float lj_d = fmaf(lj[u].x, dx[u], fmaf(lj[u].y, dy[u], lj[u].z * dz[u]));
                const float fi_d = fmaf(L.fx, dx[u], fmaf(L.fy, dy[u], L.fz * dz[u]));
                const float c1 = fmaf(P, li_fj + lj_fi, Q * fmaf(li_d, fj_d, lj_d * fi_d));
                const float w0 = fmaf(fj_d, L.lx, fmaf(li_d, fj[u].x, fmaf(fi_d, lj[u].x, lj_d * L.fx)));
                const float w1 = fmaf(fj_d, L.ly, fmaf(li_d, fj[u].y, fmaf(fi_d, lj[u].y, lj_d * L.fy)));
                const float w2 = fmaf(fj_d, L.lz, fmaf(li_d, fj[u].z, fmaf(fi_d, lj[u].z, lj_d * L.fz)));
                y0 = fmaf(c1, dx[u], fmaf(Bt, w0, y0));
                y1 = fmaf(c1, dy[u], fmaf(Bt, w1, y1));
                y2 = fmaf(c1, dz[u], fmaf(Bt, w2, y2));
                // M lam
                const float A = (TENSOR == T_OSEEN) ? rinv : fmaf(gamma, rinv3, rinv);
                const float sl = Bt * lj_d;
                z0 = fmaf(A, lj[u].x, fmaf(sl, dx[u], z0));
                z1 = fmaf(A, lj[u].y, fmaf(sl, dy[u], z1));
                z2 = fmaf(A, lj[u].z, fmaf(sl, dz[u], z2));
            }
            const float t0 = L.s0 + y0, t1 = L.s1 + y1, t2 = L.s2 + y2;
            L.c0 = (t0 - L.s0) - y0;
            L.c1 = (t1 - L.s1) - y1;
            L.c2 = (t2 - L.s2) - y2;
            L.s0 = t0;
            L.s1 = t1;
            L.s2 = t2;
            const float u0 = L.g0 + z0, u1 = L.g1 + z1, u2 = L.g2 + z2;
            L.e0 = (u0 - L.g0) - z0;
            L.e1 = (u1 - L.g1) - z1;
            L.e2 = (u2 - L.g2) - z2;
            L.g0 = u0;
            L.g1 = u1;
            L.g2 = u2;
        }
    }
    if (L.i < n) {
        const size_t base = (size_t)s * 3 * (size_t)n + (size_t)L.i;
        partial[base] = pc.alpha * ((double)L.s0 - (double)L.c0) + L.n0;
        partial[base + (size_t)n] = pc.alpha * ((double)L.s1 - (double)L.c1) + L.n1;
        partial[base + 2 * (size_t)n] = pc.alpha * ((double)L.s2 - (double)L.c2) + L.n2;
        partial_f[base] = pc.alpha * ((double)L.g0 - (double)L.e0) + L.m0;
        partial_f[base + (size_t)n] = pc.alpha * ((double)L.g1 - (double)L.e1) + L.m1;
        partial_f[base + 2 * (size_t)n] = pc.alpha * ((double)L.g2 - (double)L.e2) + L.m2;
    }
}

template <int TENSOR, int BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_adjoint_f64(const double4* __restrict__ pos, const double4* __restrict__ frc,
              const double4* __restrict__ lam, int n, int jchunk, PairConst pc,
              double* __restrict__ partial, double* __restrict__ partial_f)
{
    __shared__ double4 s_pos[BLOCK];
    __shared__ double4 s_frc[BLOCK];
    __shared__ double4 s_lam[BLOCK];
    const int tid = threadIdx.x;
    const int s = blockIdx.y;
    const int i = blockIdx.x * BLOCK + tid;
    double xi[3] = { -1.0e15, -1.0e15, -1.0e15 }, fi[3] = { 0, 0, 0 }, li[3] = { 0, 0, 0 };
    if (i < n) {
        const double4 p = pos[i], f = frc[i], l = lam[i];
        xi[0] = p.x; xi[1] = p.y; xi[2] = p.z;
        fi[0] = f.x; fi[1] = f.y; fi[2] = f.z;
        li[0] = l.x; li[1] = l.y; li[2] = l.z;
    }
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    const int jbeg = s * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const double4 far_j = make_double4(1.0e15, 1.0e15, 1.0e15, 0.0);
    const double4 zero4 = make_double4(0.0, 0.0, 0.0, 0.0);
    double4 rp = far_j, rf = zero4, rl = zero4;
    if (jbeg + tid < jend) {
        rp = pos[jbeg + tid];
        rf = frc[jbeg + tid];
        rl = lam[jbeg + tid];
    }
    for (int jt = jbeg; jt < jend; jt += BLOCK) {
        __syncthreads();
        s_pos[tid] = rp;
        s_frc[tid] = rf;
        s_lam[tid] = rl;
        __syncthreads();
        const int jn = jt + BLOCK + tid;
        rp = far_j;
        rf = zero4;
        rl = zero4;
        if (jn < jend) {
            rp = pos[jn];
            rf = frc[jn];
            rl = lam[jn];
        }
        for (int k = 0; k < BLOCK; ++k) {
            const int jg = jt + k;
            if (jg == i || jg >= n) continue;
            const double4 pj = s_pos[k], fj4 = s_frc[k], lj4 = s_lam[k];
            const double fj[3] = { fj4.x, fj4.y, fj4.z }, lj[3] = { lj4.x, lj4.y, lj4.z };
            adj_near<TENSOR>(pc, xi[0] - pj.x, xi[1] - pj.y, xi[2] - pj.z, li, fj, lj, fi, g0, g1,
                             g2);
            adj_near_mlam<TENSOR>(pc, xi[0] - pj.x, xi[1] - pj.y, xi[2] - pj.z, lj, m0, m1, m2);
        }
    }
    if (i < n) {
        const size_t base = (size_t)s * 3 * (size_t)n + (size_t)i;
        partial[base] = g0;
        partial[base + (size_t)n] = g1;
        partial[base + 2 * (size_t)n] = g2;
        partial_f[base] = m0;
        partial_f[base + (size_t)n] = m1;
        partial_f[base + 2 * (size_t)n] = m2;
    }
}

// Merge of the adjoint partials (fixed split order):
//   single product (lam64 == null): gpos = sum P;  gforce = mu0 lam4 + sum F
//   Euler loop (lam64 != null):     gforce += dt (mu0 lam_old + sum F);
//                                   lam64 = lam_old + dt sum P   (gpos unused)
template <typename P4>
__global__ void __launch_bounds__(256)
k_adjoint_merge(const double* __restrict__ pp, const double* __restrict__ pf, int S, int n,
                const P4* __restrict__ lam4, double* __restrict__ lam64, double mu0, double dt,
                double* __restrict__ gpos, double* __restrict__ gforce)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double a[3] = { 0.0, 0.0, 0.0 }, b[3] = { 0.0, 0.0, 0.0 };
    for (int s = 0; s < S; ++s) {
        const size_t base = (size_t)s * 3 * (size_t)n + (size_t)i;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            a[k] += pp[base + (size_t)k * n];
            b[k] += pf[base + (size_t)k * n];
        }
    }
    if (lam64) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const size_t e = 3 * (size_t)i + k;
            const double lo = lam64[e];
            gforce[e] += dt * (mu0 * lo + b[k]);
            lam64[e] = lo + dt * a[k];
        }
    } else {
        const P4 l = lam4[i];
        const double lv[3] = { (double)l.x, (double)l.y, (double)l.z };
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const size_t e = 3 * (size_t)i + k;
            if (gpos) gpos[e] = a[k];
            if (gforce) gforce[e] = mu0 * lv[k] + b[k];
        }
    }
}

hipError_t launch_adjoint_f32(const PairLaunch& L, int tensor, const float4* pos, const float4* frc,
                              const float4* lam, const double* x64, int n, const PairConst& pc,
                              double* partial, double* partial_f, hipStream_t st)
{
    if (L.block != 256) return hipErrorInvalidValue;
    dim3 grid((n + 255) / 256, L.splits), block(256);
    if (tensor == T_OSEEN)
        hipLaunchKernelGGL((k_adjoint_f32<T_OSEEN, 256>), grid, block, 0, st, pos, frc, lam, x64,
                           n, L.jchunk, pc, partial, partial_f);
    else
        hipLaunchKernelGGL((k_adjoint_f32<T_RPY, 256>), grid, block, 0, st, pos, frc, lam, x64, n,
                           L.jchunk, pc, partial, partial_f);
    return hipGetLastError();
}

hipError_t launch_adjoint_f64(const PairLaunch& L, int tensor, const double4* pos,
                              const double4* frc, const double4* lam, int n, const PairConst& pc,
                              double* partial, double* partial_f, hipStream_t st)
{
    if (L.block != 256) return hipErrorInvalidValue;
    dim3 grid((n + 255) / 256, L.splits), block(256);
    if (tensor == T_OSEEN)
        hipLaunchKernelGGL((k_adjoint_f64<T_OSEEN, 256>), grid, block, 0, st, pos, frc, lam, n,
                           L.jchunk, pc, partial, partial_f);
    else
        hipLaunchKernelGGL((k_adjoint_f64<T_RPY, 256>), grid, block, 0, st, pos, frc, lam, n,
                           L.jchunk, pc, partial, partial_f);
    return hipGetLastError();
}

// launch shape of the adjoint pair kernel: 256-thread groups, splits as the
// forward product's automatic choice
static PairLaunch plan_adjoint(int32_t prec, int64_t n)
{
    sd_kernel_config c = default_config(prec, n);
    PairLaunch L = shape_pair_launch((int)n, 0, 256, c.splits, 1, 0);
    L.acc = 0;
    return L;
}

// One adjoint pass: the fused pair kernel, then the merge (see k_adjoint_merge).
static sd_status adjoint_pass(const sd_params* p, int64_t n, const void* pos, const void* frc,
                              const void* lam4, const double* x64, int32_t prec, double* lam64,
                              double dt, double* gpos, double* gforce, hipStream_t hs)
{
    sd_status st;
    const PairLaunch L = plan_adjoint(prec, n);
    void* partial = nullptr;
    const size_t pb = partial_bytes(L, n);
    if ((st = ws_get(WS_ADJ_PARTIAL, 2 * pb, &partial))) return st;
    double* pp = (double*)partial;
    double* pf = (double*)((char*)partial + pb);
    const PairConst pc = pair_const(p);
    const double mu0 = 1.0 / (6.0 * M_PI * p->eta * p->a);
    hipError_t e;
    if (prec == SD_FP64) {
        e = launch_adjoint_f64(L, p->tensor, (const double4*)pos, (const double4*)frc,
                               (const double4*)lam4, (int)n, pc, pp, pf, hs);
        if (e == hipSuccess)
            hipLaunchKernelGGL((k_adjoint_merge<double4>), dim3((unsigned)((n + 255) / 256)),
                               dim3(256), 0, hs, pp, pf, L.splits, (int)n, (const double4*)lam4,
                               lam64, mu0, dt, gpos, gforce);
    } else {
        e = launch_adjoint_f32(L, p->tensor, (const float4*)pos, (const float4*)frc,
                               (const float4*)lam4, x64, (int)n, pc, pp, pf, hs);
        if (e == hipSuccess)
            hipLaunchKernelGGL((k_adjoint_merge<float4>), dim3((unsigned)((n + 255) / 256)),
                               dim3(256), 0, hs, pp, pf, L.splits, (int)n, (const float4*)lam4,
                               lam64, mu0, dt, gpos, gforce);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(SD_EDEVICE, "adjoint launch: %s", hipGetErrorString(e));
    return SD_OK;
}

}  // namespace sd

using namespace sd;

extern "C" {

sd_status mobility_adjoint(const sd_params* p, int64_t n, const void* pos, const void* force,
                           const void* lam, double* grad_pos, double* grad_force,
                           int32_t precision, void* stream)
{
    sd_status st;
    if ((st = check_params(p)) || (st = check_free_space(p, "the adjoint")) || (st = check_n(n)) ||
        (st = check_precision(precision)))
        return st;
    const size_t al = vec4_align(precision);
    if ((st = check_ptr(pos, al, "pos")) || (st = check_ptr(force, al, "force")) ||
        (st = check_ptr(lam, al, "lam")) || (st = check_ptr(grad_pos, 8, "grad_pos")))
        return st;
    if (grad_force && (uintptr_t)grad_force % 8)
        return fail(SD_EALIGN, "grad_force is not 8-byte aligned");
    return adjoint_pass(p, n, pos, force, lam, nullptr, precision, nullptr, 0.0, grad_pos,
                        grad_force, (hipStream_t)stream);
}

sd_status sd_run_adjoint(const sd_params* p, int64_t n, const double* x0, const void* force,
                         double dt, int64_t steps, int32_t precision, const double* x_checkpoints,
                         int64_t checkpoint_every, const double* grad_xN, double* grad_x0,
                         double* grad_force, void* stream)
{
    sd_status st;
    if ((st = check_params(p)) || (st = check_free_space(p, "the adjoint")) || (st = check_n(n)) ||
        (st = check_precision(precision)))
        return st;
    if ((st = check_ptr(x0, 8, "x0")) || (st = check_ptr(force, vec4_align(precision), "force")) ||
        (st = check_ptr(grad_xN, 8, "grad_xN")) || (st = check_ptr(grad_x0, 8, "grad_x0")) ||
        (st = check_ptr(grad_force, 8, "grad_force")))
        return st;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SD_EINVAL, "dt must be finite and > 0");
    if (steps < 0) return fail(SD_EINVAL, "steps must be >= 0");
    if (checkpoint_every < 1) return fail(SD_EINVAL, "checkpoint_every must be >= 1");
    if (x_checkpoints && (uintptr_t)x_checkpoints % 8)
        return fail(SD_EALIGN, "x_checkpoints is not 8-byte aligned");
    hipStream_t hs = (hipStream_t)stream;
    const size_t m = 3 * (size_t)n;
    const size_t frame = m * sizeof(double);
    const int64_t E = checkpoint_every;
    const bool f64 = precision == SD_FP64;
    const size_t rec = f64 ? 32 : 16;

    if (hipMemsetAsync(grad_force, 0, frame, hs) != hipSuccess)
        return fail(SD_EDEVICE, "hipMemsetAsync failed");
    if (hipMemcpyAsync(grad_x0, grad_xN, frame, hipMemcpyDeviceToDevice, hs) != hipSuccess)
        return fail(SD_EDEVICE, "copy failed");
    if (steps == 0) return SD_OK;

    // checkpoints of the forward pass (library-owned when the caller has none)
    const double* ck = x_checkpoints;
    if (!ck) {
        void* buf = nullptr;
        if ((st = ws_get(WS_ADJ_CKPT, frame * (size_t)(steps / E + 1), &buf))) return st;
        double* xw = (double*)buf;
        if (hipMemcpyAsync(xw, x0, frame, hipMemcpyDeviceToDevice, hs) != hipSuccess)
            return fail(SD_EDEVICE, "copy failed");
        // run from frame q to frame q+1 in place on a copy
        for (int64_t q = 0; q < steps / E; ++q) {
            double* nxt = xw + m * (size_t)(q + 1);
            if (hipMemcpyAsync(nxt, xw + m * (size_t)q, frame, hipMemcpyDeviceToDevice, hs) !=
                hipSuccess)
                return fail(SD_EDEVICE, "copy failed");
            if ((st = sd_run(p, n, nxt, force, nullptr, dt, E, q * E, SD_EULER, precision, nullptr,
                             0, stream)))
                return st;
        }
        ck = xw;
    }
    void *traj = nullptr, *pos = nullptr, *lam4 = nullptr;
    if ((st = ws_get(WS_ADJ_TRAJ, frame * (size_t)E, &traj)) ||
        (st = ws_get(WS_STAGE, rec * (size_t)n, &pos)) ||
        (st = ws_get(WS_ADJ_PACK, rec * (size_t)n, &lam4)))
        return st;
    // lam lives in grad_x0 (initialised with grad_xN above)
    double* lam = grad_x0;
    double* T = (double*)traj;
    const int64_t nseg = (steps + E - 1) / E;
    for (int64_t seg = nseg - 1; seg >= 0; --seg) {
        const int64_t k0 = seg * E;
        const int64_t k1 = std::min(steps, k0 + E);
        // x_{k0} .. x_{k1-1}: recompute the segment from its checkpoint with the
        // forward kernels (bitwise the forward pass's states)
        if (hipMemcpyAsync(T, ck + m * (size_t)seg, frame, hipMemcpyDeviceToDevice, hs) !=
            hipSuccess)
            return fail(SD_EDEVICE, "copy failed");
        for (int64_t k = k0; k + 1 < k1; ++k) {
            double* nxt = T + m * (size_t)(k - k0 + 1);
            if (hipMemcpyAsync(nxt, T + m * (size_t)(k - k0), frame, hipMemcpyDeviceToDevice, hs) !=
                hipSuccess)
                return fail(SD_EDEVICE, "copy failed");
            if ((st = sd_step(p, n, nxt, force, nullptr, nullptr, dt, k, SD_EULER, precision,
                              stream)))
                return st;
        }
        for (int64_t k = k1 - 1; k >= k0; --k) {
            const double* xk = T + m * (size_t)(k - k0);
            hipError_t e;
            e = f64 ? launch_pack_f64(xk, (double4*)pos, (int)n, hs)
                    : launch_pack_f32(xk, (float4*)pos, (int)n, hs);
            if (e == hipSuccess)
                e = f64 ? launch_pack_f64(lam, (double4*)lam4, (int)n, hs)
                        : launch_pack_f32(lam, (float4*)lam4, (int)n, hs);
            if (e != hipSuccess) return fail(SD_EDEVICE, "pack launch: %s", hipGetErrorString(e));
            // dL/dF += dt M(x_k) lam_{k+1};  lam_k = lam_{k+1} + dt d/dx [lam_{k+1} . M(x_k) F]
            if ((st = adjoint_pass(p, n, pos, force, lam4, f64 ? nullptr : xk, precision, lam, dt,
                                   nullptr, grad_force, hs)))
                return st;
        }
    }
    return SD_OK;
}

}  // extern "C"
