// pair_terms.h -- FP64 evaluation of one pair term T(d) F_j of Eq. (7a)
// (tensors of Eq. 4 and Eq. 7b, overlap form for r < 2a), shared by the
// kernels that evaluate near pairs or whole runs in FP64.
#pragma once

#include "sd_internal.h"

namespace sd {

// FP64 contribution of one near pair (d = x_i - x_j, r^2 below threshold) to
// v_i.  Returns the pair's standing against the premise r >= 2a under which
// the tensor of Eq. 4 is positive definite (Sec. 2.2): PREMISE_OK for
// r >= 2a, PREMISE_SUB2A for 0 < r < 2a, PREMISE_COINCIDENT for r = 0.
enum { PREMISE_OK = 0, PREMISE_SUB2A = 1, PREMISE_COINCIDENT = 2 };

template <int TENSOR>
__device__ __forceinline__ int near_term(const PairConst& pc, double d0, double d1, double d2,
                                         double f0, double f1, double f2, double& n0, double& n1,
                                         double& n2)
{
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (r2 == 0.0) {  // coincident distinct spheres: limit of the overlap form, else nothing
        if (TENSOR == T_RPY && pc.overlap) {
            n0 += pc.mu0 * f0;
            n1 += pc.mu0 * f1;
            n2 += pc.mu0 * f2;
        }
        return PREMISE_COINCIDENT;
    }
    const double r = sqrt(r2);
    double cI, cD;  // T = cI I + cD d d
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
    const double dF = d0 * f0 + d1 * f1 + d2 * f2;
    n0 += cI * f0 + cD * dF * d0;
    n1 += cI * f1 + cD * dF * d1;
    n2 += cI * f2 + cD * dF * d2;
    return r2 < 4.0 * pc.a * pc.a ? PREMISE_SUB2A : PREMISE_OK;
}

// v += rows s = 0, 1, ..., S-1 of a split-row array (component c of particle
// i of row s at partial[(3 s + c) n + i]), added in that order.  The loads of
// ROWS_IN_FLIGHT rows are issued before the first of their adds, so a thread
// waits for memory once per group of rows rather than once per row; the sum
// is the one of the plain loop, bit for bit.
constexpr int ROWS_IN_FLIGHT = 8;

__device__ __forceinline__ void add_split_rows(const double* __restrict__ partial, int S, int n,
                                               int i, double& v0, double& v1, double& v2)
{
    const size_t rs = 3 * (size_t)n;
    const double* p = partial + i;
    for (int s0 = 0; s0 < S; s0 += ROWS_IN_FLIGHT) {
        double a[ROWS_IN_FLIGHT][3];
#pragma unroll
        for (int u = 0; u < ROWS_IN_FLIGHT; ++u) {
            if (s0 + u < S) {
                const double* q = p + (size_t)(s0 + u) * rs;
                a[u][0] = q[0];
                a[u][1] = q[n];
                a[u][2] = q[2 * (size_t)n];
            }
        }
#pragma unroll
        for (int u = 0; u < ROWS_IN_FLIGHT; ++u) {
            if (s0 + u < S) {
                v0 += a[u][0];
                v1 += a[u][1];
                v2 += a[u][2];
            }
        }
    }
}

}  // namespace sd
