// membench.hip -- the O(N^2) memory-access micro-benchmarks of App. A on
// gfx950: N threads each read N array elements through an index map and
// accumulate them, either straight from global memory ("naive", through the
// vector and scalar caches) or through LDS tiles filled by the first wave of
// the work-group ("small tiling") or by the whole work-group ("tiling").
//
// Maps (p = 131, M = 64, the wavefront size): linear k, strided k p mod N,
// unordered (k p + j M) mod N with j the global thread id of the reading
// (naive) or loading (tiled) thread.  The indices advance by adding p mod N
// and subtracting N on overflow, so no integer division sits in the loop.
#include "sd.h"
#include "sd_host.h"
#include "sd_internal.h"

namespace sd {

constexpr unsigned MB_P = 131;
constexpr unsigned MB_M = 64;
constexpr int MB_BLOCK = 128;
constexpr int MB_WAVE = 64;

__device__ __forceinline__ float zero_of(float) { return 0.0f; }
__device__ __forceinline__ float4 zero_of(float4) { return make_float4(0.0f, 0.0f, 0.0f, 0.0f); }

// index of access k for thread j
template <int MAP>
__device__ __forceinline__ unsigned mb_start(unsigned j, unsigned N)
{
    return MAP == 2 ? (unsigned)(((unsigned long long)j * MB_M) % N) : 0u;
}

template <int MAP>
__device__ __forceinline__ unsigned mb_next(unsigned idx, unsigned step, unsigned N)
{
    if (MAP == 0) return idx + 1;
    idx += step;
    return idx >= N ? idx - N : idx;
}

template <typename T, int MAP>
__global__ void __launch_bounds__(MB_BLOCK) k_mb_naive(const T* __restrict__ in, T* __restrict__ out,
                                                       unsigned N, unsigned step)
{
    // every lane runs the loop (padding lanes j >= N too, reading in-bounds
    // elements), so a wave-uniform index stays uniform and the compiler may
    // serve it from the scalar cache
    const unsigned j = blockIdx.x * MB_BLOCK + threadIdx.x;
    T sum = j < N ? in[j] : zero_of(T());
    unsigned idx = mb_start<MAP>(j, N);
#pragma unroll 8
    for (unsigned k = 0; k < N; ++k) {
        sum += in[idx];
        idx = mb_next<MAP>(idx, step, N);
    }
    if (j < N) out[j] = sum;
}

// TILE = MB_WAVE: small tiling (the first wave loads); TILE = MB_BLOCK: tiling.
template <typename T, int MAP, int TILE>
__global__ void __launch_bounds__(MB_BLOCK) k_mb_tiled(const T* __restrict__ in, T* __restrict__ out,
                                                       unsigned N, unsigned step)
{
    __shared__ T s_data[TILE];
    const unsigned n = threadIdx.x;
    const unsigned j = blockIdx.x * MB_BLOCK + n;
    T sum = j < N ? in[j] : zero_of(T());
    // a loading thread n < TILE reads elements m + n, m = 0, TILE, 2 TILE, ...
    // advance from m to m + TILE: idx += TILE p mod N
    const unsigned tstep = (MAP == 0) ? TILE : (unsigned)(((unsigned long long)TILE * step) % N);
    unsigned idx = 0;
    if (n < TILE) {
        // index of element n for this loader
        if (MAP == 0) idx = n;
        else {
            idx = (unsigned)(((unsigned long long)n * step) % N);
            if (MAP == 2) {
                idx += mb_start<MAP>(j, N);
                if (idx >= N) idx -= N;
            }
        }
    }
    for (unsigned m = 0; m < N; m += TILE) {
        if (n < TILE) s_data[n] = (m + n < N) ? in[idx] : zero_of(T());
        __syncthreads();
        const unsigned kend = (N - m < (unsigned)TILE) ? N - m : (unsigned)TILE;
        if (kend == (unsigned)TILE) {
#pragma unroll 16
            for (unsigned k = 0; k < (unsigned)TILE; ++k) sum += s_data[k];
        } else {
            for (unsigned k = 0; k < kend; ++k) sum += s_data[k];
        }
        __syncthreads();
        if (n < TILE) {
            if (MAP == 0) idx += TILE;
            else {
                idx += tstep;
                if (idx >= N) idx -= N;
            }
        }
    }
    if (j < N) out[j] = sum;
}

template <typename T, int MAP>
static hipError_t mb_launch_t(int kind, const void* in, void* out, unsigned N, hipStream_t st)
{
    const dim3 grid((N + MB_BLOCK - 1) / MB_BLOCK), block(MB_BLOCK);
    const unsigned step = MB_P % N;
    if (kind == SD_MB_NAIVE)
        hipLaunchKernelGGL((k_mb_naive<T, MAP>), grid, block, 0, st, (const T*)in, (T*)out, N,
                           step);
    else if (kind == SD_MB_SMALLTILING)
        hipLaunchKernelGGL((k_mb_tiled<T, MAP, MB_WAVE>), grid, block, 0, st, (const T*)in,
                           (T*)out, N, step);
    else
        hipLaunchKernelGGL((k_mb_tiled<T, MAP, MB_BLOCK>), grid, block, 0, st, (const T*)in,
                           (T*)out, N, step);
    return hipGetLastError();
}

template <typename T>
static hipError_t mb_launch_m(int kind, int map, const void* in, void* out, unsigned N,
                              hipStream_t st)
{
    if (map == SD_MB_LINEAR) return mb_launch_t<T, 0>(kind, in, out, N, st);
    if (map == SD_MB_STRIDED) return mb_launch_t<T, 1>(kind, in, out, N, st);
    return mb_launch_t<T, 2>(kind, in, out, N, st);
}

}  // namespace sd

using namespace sd;

extern "C" sd_status sd_membench(int32_t kind, int32_t map, int32_t elem, int64_t n, const void* in,
                                 void* out, void* stream)
{
    sd_status st;
    if (kind < SD_MB_NAIVE || kind > SD_MB_TILING)
        return fail(SD_EINVAL, "unknown micro-benchmark kernel %d", kind);
    if (map < SD_MB_LINEAR || map > SD_MB_UNORDERED)
        return fail(SD_EINVAL, "unknown access map %d", map);
    if (elem != SD_MB_FLOAT && elem != SD_MB_FLOAT4)
        return fail(SD_EINVAL, "unknown element type %d", elem);
    if (n < 1 || n > SD_MB_MAX_N)
        return fail(SD_EINVAL, "n must be in [1, %lld] (got %lld)", (long long)SD_MB_MAX_N,
                    (long long)n);
    const size_t al = elem == SD_MB_FLOAT4 ? 16 : 4;
    if ((st = check_ptr(in, al, "in")) || (st = check_ptr(out, al, "out"))) return st;
    hipStream_t hs = (hipStream_t)stream;
    const hipError_t e = elem == SD_MB_FLOAT4
                             ? mb_launch_m<float4>(kind, map, in, out, (unsigned)n, hs)
                             : mb_launch_m<float>(kind, map, in, out, (unsigned)n, hs);
    if (e != hipSuccess) return fail(SD_EDEVICE, "micro-benchmark launch: %s", hipGetErrorString(e));
    return SD_OK;
}
