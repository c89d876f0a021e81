// integrate.hip -- O(N) kernels of the time loop (Sec. 3.1, step 1) and small
// helpers: FP64 -> FP32 staging of positions, split merge fused with the
// Euler / AB2 position update, packing and axpy for the adjoint loop.
#include "pair_terms.h"
#include "sd_internal.h"

namespace sd {

// Fixed-point coordinate of a periodic box (q = x 2^32 / Lb mod 2^32, see
// PairConst), returned as the bits of a float record.  qs = 2^32 / Lb.
__device__ __forceinline__ float fixed_coord(double x, double qs)
{
    const long long t = (long long)rint(x * qs);
    return __uint_as_float((unsigned int)(unsigned long long)t);
}

// FP32 record of a position: plain FP32 (qs = 0) or fixed point (qs > 0).
__device__ __forceinline__ void put_pos(float4* p, int i, double a, double b, double c, double qs)
{
    if (qs > 0.0)
        p[i] = make_float4(fixed_coord(a, qs), fixed_coord(b, qs), fixed_coord(c, qs), 0.0f);
    else
        p[i] = make_float4((float)a, (float)b, (float)c, 0.0f);
}
__device__ __forceinline__ void put_pos(double4* p, int i, double a, double b, double c, double)
{
    p[i] = make_double4(a, b, c, 0.0);
}

template <typename P4>
__global__ void __launch_bounds__(256) k_stage(const double* __restrict__ x, P4* __restrict__ pos,
                                               int n, double qs)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    put_pos(pos, i, x[3 * (size_t)i], x[3 * (size_t)i + 1], x[3 * (size_t)i + 2], qs);
}

__global__ void __launch_bounds__(256) k_stage_q_from_f32(const float4* __restrict__ pos,
                                                          float4* __restrict__ q, int n, double qs)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float4 p = pos[i];
    put_pos(q, i, (double)p.x, (double)p.y, (double)p.z, qs);
}

// v_k = mu0 F + sum_s partial_s (the same order as k_merge), then
//   mode 0: x += dt v                       (Euler)
//   mode 1: x += dt v,  v_prev = v           (first AB2 step)
//   mode 2: x += dt (3/2 v - 1/2 v_prev), v_prev = v   (AB2)
// and the staged copy of the new positions for the next pair kernel.
template <typename F4, typename P4>
__global__ void __launch_bounds__(256)
k_merge_integrate(const double* __restrict__ partial, int S, int n, const F4* __restrict__ frc,
                  double mu0, double* __restrict__ x, double* __restrict__ v_prev,
                  double* __restrict__ v_out, double dt, int mode, P4* __restrict__ pos_next,
                  double qs)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const F4 f = frc[i];
    double v[3] = { mu0 * (double)f.x, mu0 * (double)f.y, mu0 * (double)f.z };
    add_split_rows(partial, S, n, i, v[0], v[1], v[2]);
    double xn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const size_t e = 3 * (size_t)i + k;
        const double inc = (mode == 2) ? (1.5 * v[k] - 0.5 * v_prev[e]) : v[k];
        xn[k] = x[e] + dt * inc;
        x[e] = xn[k];
        if (mode != 0) v_prev[e] = v[k];
        if (v_out) v_out[e] = v[k];
    }
    if (pos_next) put_pos(pos_next, i, xn[0], xn[1], xn[2], qs);
}

__global__ void __launch_bounds__(256) k_sum_partials(const double* __restrict__ partial, int S,
                                                      int n, double* __restrict__ out,
                                                      double scale, int accumulate)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double g[3] = { 0.0, 0.0, 0.0 };
    add_split_rows(partial, S, n, i, g[0], g[1], g[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const size_t e = 3 * (size_t)i + k;
        out[e] = accumulate ? out[e] + scale * g[k] : scale * g[k];
    }
}

template <typename P4>
__global__ void __launch_bounds__(256) k_pack(const double* __restrict__ v, P4* __restrict__ out,
                                              int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    put_pos(out, i, v[3 * (size_t)i], v[3 * (size_t)i + 1], v[3 * (size_t)i + 2], 0.0);
}

__global__ void __launch_bounds__(256) k_axpy(double s, const double* __restrict__ x,
                                              double* __restrict__ y, int64_t m)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < m) y[k] += s * x[k];
}

__global__ void __launch_bounds__(64) k_fill_i32(int32_t* __restrict__ p, int32_t value, int count)
{
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k < count) p[k] = value;
}

// out = (1/n) sum_i v_i in a fixed order, in two launches: G = mean_groups(n)
// work-groups each sum a contiguous range of ceil(n / G) particles (lane t:
// particles t, t + 256, ... of the range in order, then a fixed-shape tree
// over the 256 lanes) into partial[c G + g]; one work-group then sums the G
// partials the same way.  The grouping depends on n only, so the result does
// not depend on the device or on the scheduling of the work-groups.
int64_t mean_groups(int64_t n)
{
    const int64_t g = (n + 1023) / 1024;
    return g < 1 ? 1 : (g > 1024 ? 1024 : g);
}

// the three lane sums of a 256-lane work-group -> lane 0, fixed shape
__device__ __forceinline__ void tree3(double (&red)[3][256], int t, double a0, double a1,
                                      double a2)
{
    red[0][t] = a0;
    red[1][t] = a1;
    red[2][t] = a2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] += red[1][t + w];
            red[2][t] += red[2][t + w];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_mean_partial(const double* __restrict__ v, int64_t n,
                                                      int64_t chunk, int groups,
                                                      double* __restrict__ partial)
{
    __shared__ double red[3][256];
    const int t = threadIdx.x, g = blockIdx.x;
    const int64_t i0 = (int64_t)g * chunk;
    const int64_t i1 = i0 + chunk < n ? i0 + chunk : n;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t i = i0 + t; i < i1; i += 256) {
        a0 += v[3 * i];
        a1 += v[3 * i + 1];
        a2 += v[3 * i + 2];
    }
    tree3(red, t, a0, a1, a2);
    if (t < 3) partial[(int64_t)t * groups + g] = red[t][0];
}

__global__ void __launch_bounds__(256) k_mean_final(const double* __restrict__ partial,
                                                    int groups, int64_t n,
                                                    double* __restrict__ out)
{
    __shared__ double red[3][256];
    const int t = threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int k = t; k < groups; k += 256) {
        a0 += partial[k];
        a1 += partial[groups + k];
        a2 += partial[2 * groups + k];
    }
    tree3(red, t, a0, a1, a2);
    if (t < 3) out[t] = red[t][0] / (double)n;
}

hipError_t launch_mean_vector(const double* v, int64_t n, double* out, double* partial,
                              hipStream_t st)
{
    const int64_t g = mean_groups(n);
    const int64_t chunk = (n + g - 1) / g;
    hipLaunchKernelGGL(k_mean_partial, dim3((unsigned)g), dim3(256), 0, st, v, n, chunk, (int)g,
                       partial);
    hipLaunchKernelGGL(k_mean_final, dim3(1), dim3(256), 0, st, partial, (int)g, n, out);
    return hipGetLastError();
}

static inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// 2^32 / Lb, the fixed-point scale of a periodic box (0 in free space)
static inline double q_scale(double box) { return box > 0.0 ? 4294967296.0 / box : 0.0; }

hipError_t launch_stage_f32(const double* x, float4* pos, int n, double box, hipStream_t st)
{
    hipLaunchKernelGGL((k_stage<float4>), grid_for(n), dim3(256), 0, st, x, pos, n,
                       q_scale(box));
    return hipGetLastError();
}

hipError_t launch_stage_f64(const double* x, double4* pos, int n, hipStream_t st)
{
    hipLaunchKernelGGL((k_stage<double4>), grid_for(n), dim3(256), 0, st, x, pos, n, 0.0);
    return hipGetLastError();
}

hipError_t launch_stage_q_from_f32(const float4* pos, float4* q, int n, double box,
                                   hipStream_t st)
{
    hipLaunchKernelGGL(k_stage_q_from_f32, grid_for(n), dim3(256), 0, st, pos, q, n,
                       q_scale(box));
    return hipGetLastError();
}

hipError_t launch_merge_integrate_f32(const double* partial, int splits, int n, const float4* frc,
                                      double mu0, double* x, double* v_prev, double* v_out,
                                      double dt, int mode, float4* pos_next, double box,
                                      hipStream_t st)
{
    hipLaunchKernelGGL((k_merge_integrate<float4, float4>), grid_for(n), dim3(256), 0, st, partial,
                       splits, n, frc, mu0, x, v_prev, v_out, dt, mode, pos_next, q_scale(box));
    return hipGetLastError();
}

hipError_t launch_merge_integrate_f64(const double* partial, int splits, int n, const double4* frc,
                                      double mu0, double* x, double* v_prev, double* v_out,
                                      double dt, int mode, double4* pos_next, hipStream_t st)
{
    hipLaunchKernelGGL((k_merge_integrate<double4, double4>), grid_for(n), dim3(256), 0, st,
                       partial, splits, n, frc, mu0, x, v_prev, v_out, dt, mode, pos_next, 0.0);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partial, int splits, int n, double* out, double scale,
                               int accumulate, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_partials, grid_for(n), dim3(256), 0, st, partial, splits, n, out,
                       scale, accumulate);
    return hipGetLastError();
}

hipError_t launch_pack_f32(const double* v, float4* out, int n, hipStream_t st)
{
    hipLaunchKernelGGL((k_pack<float4>), grid_for(n), dim3(256), 0, st, v, out, n);
    return hipGetLastError();
}

hipError_t launch_pack_f64(const double* v, double4* out, int n, hipStream_t st)
{
    hipLaunchKernelGGL((k_pack<double4>), grid_for(n), dim3(256), 0, st, v, out, n);
    return hipGetLastError();
}

hipError_t launch_axpy(double s, const double* x, double* y, int64_t m, hipStream_t st)
{
    hipLaunchKernelGGL(k_axpy, grid_for(m), dim3(256), 0, st, s, x, y, m);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t value, int count, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_i32, dim3((count + 63) / 64), dim3(64), 0, st, p, value, count);
    return hipGetLastError();
}

}  // namespace sd
