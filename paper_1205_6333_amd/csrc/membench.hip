// membench.hip -- the O(N^2) memory-access micro-benchmarks of App. A on
// gfx950: N threads each read N array elements through an index map and
// accumulate them, either straight from global memory ("naive", through the
// vector and scalar caches) or through LDS tiles filled by the first wave of
// the work-group ("small tiling") or by the whole work-group ("tiling").
//
// Maps (p = 131, M = 64, the wavefront size): linear k, strided k p mod N,
// unordered (k p + g M) mod N with g the global thread id of the reading
// (direct) or fetching (staged) thread.  The indices advance by adding a
// precomputed increment mod N and subtracting N on overflow, so no integer
// division sits in the loop.
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

// Position in the index map of App. A: element k of the sequence read by the
// thread with global id `owner` (the reader for the direct kernel, the loader
// for the staged ones).  Linear: k; strided: k p mod N; unordered:
// (k p + owner M) mod N.  advance(d) moves from k to k + d, with d p mod N
// precomputed, by one add and one conditional subtract.
template <int MAP>
struct MapCursor {
    unsigned at;     // current index into the array
    unsigned hop;    // index increment of one advance (mod N)
    unsigned N;
    __device__ MapCursor(unsigned k0, unsigned owner, unsigned stride, unsigned N_)
        : N(N_)
    {
        if (MAP == 0) {   // k itself: the increment stays a compile-time constant
            at = k0;
            hop = stride;
            return;
        }
        const unsigned long long p = MB_P % N_;
        const unsigned long long base = MAP == 2 ? (unsigned long long)owner * MB_M : 0ull;
        at = (unsigned)(((unsigned long long)k0 * p + base) % N_);
        hop = (unsigned)(((unsigned long long)stride * p) % N_);
    }
    __device__ __forceinline__ void advance()
    {
        at += hop;
        // the linear map does not wrap within the N elements of a sequence
        // (a staged loader's index past N is not read), and without the
        // compare the compiler sees consecutive indices and merges their
        // wave-uniform loads
        if (MAP != 0 && at >= N) at -= N;
    }
};

// Direct ("naive"): every thread sums its own element and then the whole
// map sequence k = 0 .. N-1 straight from memory.  Threads past N run the
// loop too (on in-bounds indices), so that indices common to a wave stay
// wave-uniform and may be served by the scalar cache.
template <typename T, int MAP>
__global__ void __launch_bounds__(MB_BLOCK) k_mb_naive(const T* __restrict__ in, T* __restrict__ out,
                                                       unsigned N)
{
    const unsigned me = blockIdx.x * MB_BLOCK + threadIdx.x;
    T acc = me < N ? in[me] : zero_of(T());
    MapCursor<MAP> cur(0u, me, 1u, N);
#pragma unroll 8
    for (unsigned k = 0; k < N; ++k) {
        acc += in[cur.at];
        cur.advance();
    }
    if (me < N) out[me] = acc;
}

// Staged ("small tiling" with LOADERS = one wave, "tiling" with LOADERS = the
// work-group): the sequence is read in tiles of LOADERS elements, loader t
// fetching element c LOADERS + t of tile c through ITS OWN map (unordered:
// offset by the loader's global id), and every thread of the work-group sums
// the tile from LDS in order.  Two LDS buffers: tile c + 1 is fetched while
// tile c is summed, one barrier per tile.
template <typename T, int MAP, int LOADERS>
__global__ void __launch_bounds__(MB_BLOCK) k_mb_tiled(const T* __restrict__ in, T* __restrict__ out,
                                                       unsigned N)
{
    __shared__ T stage[2][LOADERS];
    const unsigned lt = threadIdx.x;
    const unsigned me = blockIdx.x * MB_BLOCK + lt;
    const bool loader = lt < (unsigned)LOADERS;
    T acc = me < N ? in[me] : zero_of(T());
    MapCursor<MAP> cur(loader ? lt : 0u, me, LOADERS, N);
    const unsigned tiles = (N + LOADERS - 1) / LOADERS;
    auto fetch = [&](unsigned c, int b) {
        if (loader) {
            stage[b][lt] = c * LOADERS + lt < N ? in[cur.at] : zero_of(T());
            cur.advance();
        }
    };
    fetch(0u, 0);
    __syncthreads();
    for (unsigned c = 0; c < tiles; ++c) {
        const int b = (int)(c & 1u);
        if (c + 1 < tiles) fetch(c + 1, b ^ 1);
        const unsigned cnt = N - c * LOADERS < (unsigned)LOADERS ? N - c * LOADERS : LOADERS;
        if (cnt == (unsigned)LOADERS) {
#pragma unroll 16
            for (unsigned e = 0; e < (unsigned)LOADERS; ++e) acc += stage[b][e];
        } else {
            for (unsigned e = 0; e < cnt; ++e) acc += stage[b][e];
        }
        __syncthreads();
    }
    if (me < N) out[me] = acc;
}

template <typename T, int MAP>
static hipError_t mb_launch_t(int kind, const void* in, void* out, unsigned N, hipStream_t st)
{
    const dim3 grid((N + MB_BLOCK - 1) / MB_BLOCK), block(MB_BLOCK);
    if (kind == SD_MB_NAIVE)
        hipLaunchKernelGGL((k_mb_naive<T, MAP>), grid, block, 0, st, (const T*)in, (T*)out, N);
    else if (kind == SD_MB_SMALLTILING)
        hipLaunchKernelGGL((k_mb_tiled<T, MAP, MB_WAVE>), grid, block, 0, st, (const T*)in,
                           (T*)out, N);
    else
        hipLaunchKernelGGL((k_mb_tiled<T, MAP, MB_BLOCK>), grid, block, 0, st, (const T*)in,
                           (T*)out, N);
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
