// lubrication.hip -- the lubrication correction of Eq. (8) folded into the
// forces with the previous step's velocities (Sec. 3.1, step 2):
//   F_i = F_ext,i - sum'_j zeta(r_i - r_j) (v_i - v_j),
//   mu0 zeta(r) = [1/(4s) - 9/40 log s] rhat rhat - 1/6 log s (I - rhat rhat),
//   s = r/a - 2 < s_cut (Sec. 2.3: s_cut = 1), clamped to s >= s_min.
// The primed sum runs over close pairs only, found with a cell list rebuilt on
// the device every step (cells of side >= (2 + s_cut) a; the grid is derived
// from the bounding box on the device, so a step needs no host round trip).
// Cells are filled with integer atomics and then sorted by particle index, so
// the summation order, and hence the result, is deterministic.  In a periodic
// cubic box the grid tiles the box, cell neighbours wrap around, and each pair
// interacts through its nearest image only.  All of it is
// O(N x neighbours) FP64 work next to the O(N^2) mobility product.
#include "sd.h"
#include "sd_host.h"
#include "sd_internal.h"

#include <algorithm>
#include <cmath>

namespace sd {

constexpr int LUB_MAX_CELLS = 1 << 21;   // cap of the cell grid (cells grow beyond the cutoff if needed)
constexpr int SCAN_B = 2048;                          // cells per scan block (256 threads x 8)
constexpr int SCAN_NB = LUB_MAX_CELLS / SCAN_B;       // 1024 scan blocks at most
constexpr int BBOX_NB = 1024;                         // bounding-box partials at most

struct CellGrid {
    double lo[3];
    double h;        // cell side
    double box;      // periodic cubic box side, 0 = free space
    int dims[3];
    int ncell;
};

struct LubConst {
    double a, mu0, s_cut, s_min, rcut2;
    PairConst pc;    // box for the nearest image
};

// Bounding box, stage 1: work-group b reduces particles [b chunk, (b+1) chunk)
// to part[b] = (lo xyz, hi xyz).  min / max are exact, so the result does not
// depend on the reduction order.
__global__ void __launch_bounds__(256) k_lub_bbox(const double* __restrict__ x, int n, int chunk,
                                                  double* __restrict__ part)
{
    __shared__ double lo[3][256], hi[3][256];
    const int t = threadIdx.x;
    const int b0 = blockIdx.x * chunk, b1 = min(n, b0 + chunk);
    double l[3] = { 1e300, 1e300, 1e300 }, u[3] = { -1e300, -1e300, -1e300 };
    for (int i = b0 + t; i < b1; i += 256)
        for (int k = 0; k < 3; ++k) {
            const double v = x[3 * (size_t)i + k];
            l[k] = fmin(l[k], v);
            u[k] = fmax(u[k], v);
        }
    for (int k = 0; k < 3; ++k) {
        lo[k][t] = l[k];
        hi[k][t] = u[k];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 3; ++k) {
                lo[k][t] = fmin(lo[k][t], lo[k][t + w]);
                hi[k][t] = fmax(hi[k][t], hi[k][t + w]);
            }
        __syncthreads();
    }
    if (t < 3) {
        part[6 * blockIdx.x + t] = lo[t][0];
        part[6 * blockIdx.x + 3 + t] = hi[t][0];
    }
}

// Bounding box, stage 2 (one work-group) -> cell grid; free space reduces the
// nparts partials, a periodic box tiles the cube.
__global__ void __launch_bounds__(256) k_lub_grid(const double* __restrict__ part, int nparts,
                                                  double hmin, double box,
                                                  CellGrid* __restrict__ g)
{
    if (box > 0.0) {  // periodic: the grid tiles the box, cells no smaller than hmin
        if (threadIdx.x == 0) {
            int d = (int)floor(box / hmin);
            d = d < 1 ? 1 : (d > 128 ? 128 : d);  // 128^3 <= LUB_MAX_CELLS
            for (int k = 0; k < 3; ++k) {
                g->lo[k] = 0.0;
                g->dims[k] = d;
            }
            g->h = box / d;
            g->box = box;
            g->ncell = d * d * d;
        }
        return;
    }
    __shared__ double lo[3][256], hi[3][256];
    const int t = threadIdx.x;
    double l[3] = { 1e300, 1e300, 1e300 }, u[3] = { -1e300, -1e300, -1e300 };
    for (int b = t; b < nparts; b += 256)
        for (int k = 0; k < 3; ++k) {
            l[k] = fmin(l[k], part[6 * b + k]);
            u[k] = fmax(u[k], part[6 * b + 3 + k]);
        }
    for (int k = 0; k < 3; ++k) {
        lo[k][t] = l[k];
        hi[k][t] = u[k];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 3; ++k) {
                lo[k][t] = fmin(lo[k][t], lo[k][t + w]);
                hi[k][t] = fmax(hi[k][t], hi[k][t + w]);
            }
        __syncthreads();
    }
    if (t == 0) {
        double ext[3], h = hmin;
        for (int k = 0; k < 3; ++k) {
            ext[k] = hi[k][0] - lo[k][0];
            // non-finite coordinates (NaN / Inf inputs) collapse that axis to one cell
            if (!(ext[k] >= 0.0) || !(ext[k] < 1e300)) ext[k] = 0.0;
            if (!(lo[k][0] > -1e300)) lo[k][0] = 0.0;
        }
        // grow the cell until the grid fits the cap (bounded: 1.25^400 covers any
        // finite extent)
        for (int it = 0; it < 400; ++it) {
            double cells = 1.0;
            for (int k = 0; k < 3; ++k) cells *= floor(ext[k] / h) + 1.0;
            if (cells <= (double)LUB_MAX_CELLS) break;
            h *= 1.25;
        }
        int nc = 1;
        for (int k = 0; k < 3; ++k) {
            g->lo[k] = lo[k][0];
            g->dims[k] = (int)floor(ext[k] / h) + 1;
            nc *= g->dims[k];
        }
        g->h = h;
        g->box = 0.0;
        g->ncell = nc;
    }
}

__device__ __forceinline__ int cell_coord(double v, double lo, double h, int dim, double box)
{
    if (box > 0.0) v -= box * floor(v / box);  // wrap into [0, box)
    int c = (int)floor((v - lo) / h);
    return c < 0 ? 0 : (c >= dim ? dim - 1 : c);
}

// Distinct neighbour cells of cell c along one axis: c-1, c, c+1, clipped to
// the grid in free space, wrapped (and de-duplicated on grids narrower than
// three cells) in a periodic box.  Returns the count.
__device__ __forceinline__ int axis_neighbours(int c, int dim, bool periodic, int (&out)[3])
{
    int m = 0;
    if (periodic) {
        if (dim < 3) {
            for (int k = 0; k < dim; ++k) out[m++] = k;
        } else {
            out[m++] = c == 0 ? dim - 1 : c - 1;
            out[m++] = c;
            out[m++] = c == dim - 1 ? 0 : c + 1;
        }
    } else {
        for (int k = c - 1; k <= c + 1; ++k)
            if (k >= 0 && k < dim) out[m++] = k;
    }
    return m;
}

__global__ void __launch_bounds__(256) k_lub_count(const double* __restrict__ x, int n,
                                                   const CellGrid* __restrict__ g,
                                                   int* __restrict__ cid, int* __restrict__ count)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double h = g->h;
    const int cx = cell_coord(x[3 * (size_t)i], g->lo[0], h, g->dims[0], g->box);
    const int cy = cell_coord(x[3 * (size_t)i + 1], g->lo[1], h, g->dims[1], g->box);
    const int cz = cell_coord(x[3 * (size_t)i + 2], g->lo[2], h, g->dims[2], g->box);
    const int c = (cz * g->dims[1] + cy) * g->dims[0] + cx;
    cid[i] = c;
    atomicAdd(&count[c], 1);
}

// Exclusive scan of the cell counts in three passes: per-block sums of SCAN_B
// cells, a scan of the (at most SCAN_NB) block sums in one work-group, then
// each block scans its cells from its offset.  start[ncell] = n; the counts
// are reset to zero for use as scatter cursors.  Integer sums: the result is
// exact and independent of the order.
__device__ __forceinline__ int block_exclusive_scan_256(int v, int* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {
        const int a = t >= w ? sh[t - w] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    const int incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(256) k_lub_scan_sums(const int* __restrict__ count,
                                                       const CellGrid* __restrict__ g,
                                                       int* __restrict__ bsum)
{
    __shared__ int sh[256];
    const int nc = g->ncell;
    const int c0 = blockIdx.x * SCAN_B + threadIdx.x * (SCAN_B / 256);
    if (blockIdx.x * SCAN_B >= nc) return;   // uniform per block
    int v = 0;
    for (int c = c0; c < c0 + SCAN_B / 256; ++c)
        if (c < nc) v += count[c];
    const int ex = block_exclusive_scan_256(v, sh);
    if (threadIdx.x == 255) bsum[blockIdx.x] = ex + v;
}

__global__ void __launch_bounds__(1024) k_lub_scan_top(int* __restrict__ bsum,
                                                       const CellGrid* __restrict__ g)
{
    __shared__ int sh[1024];
    const int t = threadIdx.x;
    const int nb = (g->ncell + SCAN_B - 1) / SCAN_B;
    const int v = t < nb ? bsum[t] : 0;
    sh[t] = v;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {
        const int a = t >= w ? sh[t - w] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    if (t < nb) bsum[t] = sh[t] - v;   // exclusive offsets
}

__global__ void __launch_bounds__(256) k_lub_scan_apply(int* __restrict__ count,
                                                        int* __restrict__ start,
                                                        const int* __restrict__ boff,
                                                        const CellGrid* __restrict__ g, int n)
{
    __shared__ int sh[256];
    const int nc = g->ncell;
    if (blockIdx.x * SCAN_B >= nc) return;   // uniform per block
    const int c0 = blockIdx.x * SCAN_B + threadIdx.x * (SCAN_B / 256);
    int v = 0;
    for (int c = c0; c < c0 + SCAN_B / 256; ++c)
        if (c < nc) v += count[c];
    int run = boff[blockIdx.x] + block_exclusive_scan_256(v, sh);
    for (int c = c0; c < c0 + SCAN_B / 256; ++c)
        if (c < nc) {
            const int k = count[c];
            start[c] = run;
            run += k;
            count[c] = 0;
        }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[nc] = n;
}

__global__ void __launch_bounds__(256) k_lub_scatter(const int* __restrict__ cid, int n,
                                                     const int* __restrict__ start,
                                                     int* __restrict__ cursor,
                                                     int* __restrict__ order)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = cid[i];
    order[start[c] + atomicAdd(&cursor[c], 1)] = i;
}

// each cell's members in ascending particle index (cells hold a handful)
__global__ void __launch_bounds__(256) k_lub_sort(const int* __restrict__ start,
                                                  int* __restrict__ order,
                                                  const CellGrid* __restrict__ g)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= g->ncell) return;
    const int b = start[c], e = start[c + 1];
    for (int k = b + 1; k < e; ++k) {
        const int v = order[k];
        int m = k - 1;
        while (m >= b && order[m] > v) {
            order[m + 1] = order[m];
            --m;
        }
        order[m + 1] = v;
    }
}

__global__ void __launch_bounds__(256)
k_lub_force(const double* __restrict__ x, const double* __restrict__ v,
            const double* __restrict__ f_ext, int n, const CellGrid* __restrict__ g,
            const int* __restrict__ start, const int* __restrict__ order, LubConst lc,
            double* __restrict__ f_out, float4* __restrict__ rec32, double4* __restrict__ rec64)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double xi[3] = { x[3 * (size_t)i], x[3 * (size_t)i + 1], x[3 * (size_t)i + 2] };
    const double vi[3] = { v[3 * (size_t)i], v[3 * (size_t)i + 1], v[3 * (size_t)i + 2] };
    const double h = g->h;
    const int dims[3] = { g->dims[0], g->dims[1], g->dims[2] };
    const bool per = g->box > 0.0;
    int nb[3][3], nn[3];
    for (int k = 0; k < 3; ++k)
        nn[k] = axis_neighbours(cell_coord(xi[k], g->lo[k], h, dims[k], g->box), dims[k], per,
                                nb[k]);
    double acc[3] = { 0.0, 0.0, 0.0 };
    for (int iz = 0; iz < nn[2]; ++iz) {
        const int z = nb[2][iz];
        for (int iy = 0; iy < nn[1]; ++iy) {
            const int y = nb[1][iy];
            for (int ix = 0; ix < nn[0]; ++ix) {
                const int xx = nb[0][ix];
                const int c = (z * dims[1] + y) * dims[0] + xx;
                for (int k = start[c]; k < start[c + 1]; ++k) {
                    const int j = order[k];
                    if (j == i) continue;
                    double d[3] = { xi[0] - x[3 * (size_t)j], xi[1] - x[3 * (size_t)j + 1],
                                    xi[2] - x[3 * (size_t)j + 2] };
                    nearest_image_d(lc.pc, d[0], d[1], d[2]);
                    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    if (!(r2 < lc.rcut2) || r2 == 0.0) continue;
                    const double r = sqrt(r2);
                    double s = r / lc.a - 2.0;
                    if (s >= lc.s_cut) continue;
                    if (s < lc.s_min) s = lc.s_min;
                    const double ls = log(s);
                    const double cP = (1.0 / (4.0 * s) - 9.0 / 40.0 * ls) / lc.mu0;
                    const double cT = (-1.0 / 6.0 * ls) / lc.mu0;
                    const double dv[3] = { vi[0] - v[3 * (size_t)j], vi[1] - v[3 * (size_t)j + 1],
                                           vi[2] - v[3 * (size_t)j + 2] };
                    const double hd = (d[0] * dv[0] + d[1] * dv[1] + d[2] * dv[2]) / r;  // rhat . dv
                    for (int k3 = 0; k3 < 3; ++k3) {
                        const double nrm = hd * d[k3] / r;                             // (rhat rhat dv)_k
                        acc[k3] -= cP * nrm + cT * (dv[k3] - nrm);
                    }
                }
            }
        }
    }
    double fo[3];
    for (int k = 0; k < 3; ++k) fo[k] = (f_ext ? f_ext[3 * (size_t)i + k] : 0.0) + acc[k];
    // the FP64 vector and/or the force record the pair kernel reads
    if (f_out)
        for (int k = 0; k < 3; ++k) f_out[3 * (size_t)i + k] = fo[k];
    if (rec32) rec32[i] = make_float4((float)fo[0], (float)fo[1], (float)fo[2], 0.0f);
    if (rec64) rec64[i] = make_double4(fo[0], fo[1], fo[2], 0.0);
}

// Library workspace of the cell list: grid | bbox partials f64[6 BBOX_NB] |
// block sums int[SCAN_NB] | cid[n] | order[n] | count[MAX] | start[MAX+1]
static size_t lub_ws_bytes(int64_t n)
{
    return 256 + 48 * (size_t)BBOX_NB + 4 * (size_t)SCAN_NB + 4 * (size_t)n * 2 +
           4 * ((size_t)LUB_MAX_CELLS * 2 + 1) + 256;
}

// f_out (f64[3n]), rec32 (f32x4[n]) and rec64 (f64x4[n]) receive the forces
// when non-null.
sd_status lub_forces_impl(const sd_params* p, const sd_lub* lub, int64_t n, const double* x,
                          const double* v, const double* f_ext, double* f_out, float4* rec32,
                          double4* rec64, hipStream_t hs)
{
    sd_status st;
    void* buf = nullptr;
    if ((st = ws_get(WS_LUB, lub_ws_bytes(n), &buf))) return st;
    char* q = (char*)buf;
    CellGrid* g = (CellGrid*)q;
    q += 256;
    double* bbox = (double*)q;
    q += 48 * (size_t)BBOX_NB;
    int* bsum = (int*)q;
    q += 4 * (size_t)SCAN_NB;
    int* cid = (int*)q;
    q += 4 * (size_t)n;
    int* order = (int*)q;
    q += 4 * (size_t)n;
    int* count = (int*)q;
    q += 4 * (size_t)LUB_MAX_CELLS;
    int* start = (int*)q;
    const int nn = (int)n;
    const dim3 gp((unsigned)((n + 255) / 256));
    hipError_t e = launch_fill_i32(count, 0, LUB_MAX_CELLS, hs);
    if (e != hipSuccess) return fail(SD_EDEVICE, "fill launch: %s", hipGetErrorString(e));
    int nparts = 0;
    if (!(box_side(p) > 0.0)) {  // free space: bounding box of the particles
        nparts = (int)std::min<int64_t>(BBOX_NB, std::max<int64_t>(1, (n + 4095) / 4096));
        const int chunk = (int)((n + nparts - 1) / nparts);
        hipLaunchKernelGGL(k_lub_bbox, dim3(nparts), dim3(256), 0, hs, x, nn, chunk, bbox);
    }
    hipLaunchKernelGGL(k_lub_grid, dim3(1), dim3(256), 0, hs, bbox, nparts,
                       (2.0 + lub->s_cut) * p->a, box_side(p), g);
    hipLaunchKernelGGL(k_lub_count, gp, dim3(256), 0, hs, x, nn, g, cid, count);
    hipLaunchKernelGGL(k_lub_scan_sums, dim3(SCAN_NB), dim3(256), 0, hs, count, g, bsum);
    hipLaunchKernelGGL(k_lub_scan_top, dim3(1), dim3(1024), 0, hs, bsum, g);
    hipLaunchKernelGGL(k_lub_scan_apply, dim3(SCAN_NB), dim3(256), 0, hs, count, start, bsum, g,
                       nn);
    hipLaunchKernelGGL(k_lub_scatter, gp, dim3(256), 0, hs, cid, nn, start, count, order);
    hipLaunchKernelGGL(k_lub_sort, dim3(LUB_MAX_CELLS / 256), dim3(256), 0, hs, start, order, g);
    LubConst lc;
    lc.a = p->a;
    lc.mu0 = 1.0 / (6.0 * M_PI * p->eta * p->a);
    lc.s_cut = lub->s_cut;
    lc.s_min = lub->s_min;
    const double rc = (2.0 + lub->s_cut) * p->a;
    lc.rcut2 = rc * rc;
    lc.pc = pair_const(p);
    hipLaunchKernelGGL(k_lub_force, gp, dim3(256), 0, hs, x, v, f_ext, nn, g, start, order, lc,
                       f_out, rec32, rec64);
    if ((e = hipGetLastError()) != hipSuccess)
        return fail(SD_EDEVICE, "lubrication launch: %s", hipGetErrorString(e));
    return SD_OK;
}

sd_status check_lub(const sd_lub* lub)
{
    if (!lub) return fail(SD_EINVAL, "lub is NULL");
    if (!(lub->s_cut > 0.0) || !std::isfinite(lub->s_cut))
        return fail(SD_EINVAL, "s_cut must be finite and > 0");
    if (!(lub->s_min > 0.0) || !(lub->s_min < lub->s_cut))
        return fail(SD_EINVAL, "s_min must be in (0, s_cut)");
    return SD_OK;
}

}  // namespace sd

using namespace sd;

extern "C" {

sd_status lubrication_forces(const sd_params* p, const sd_lub* lub, int64_t n, const double* x,
                             const double* v, const double* f_ext, double* f_out, void* stream)
{
    sd_status st;
    if ((st = check_params(p)) || (st = check_lub(lub)) || (st = check_n(n))) return st;
    if ((st = check_ptr(x, 8, "x")) || (st = check_ptr(v, 8, "v")) ||
        (st = check_ptr(f_out, 8, "f_out")))
        return st;
    if (f_ext && (uintptr_t)f_ext % 8) return fail(SD_EALIGN, "f_ext is not 8-byte aligned");
    return lub_forces_impl(p, lub, n, x, v, f_ext, f_out, nullptr, nullptr, (hipStream_t)stream);
}

sd_status sd_run_lub(const sd_params* p, const sd_lub* lub, int64_t n, double* x,
                     const double* f_ext, double* v_prev, double dt, int64_t steps, int64_t step0,
                     int32_t integrator, int32_t precision, void* stream)
{
    sd_status st;
    if ((st = check_params(p)) || (st = check_lub(lub)) || (st = check_n(n)) ||
        (st = check_precision(precision)))
        return st;
    if ((st = check_ptr(x, 8, "x")) || (st = check_ptr(f_ext, 8, "f_ext")) ||
        (st = check_ptr(v_prev, 8, "v_prev")))
        return st;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SD_EINVAL, "dt must be finite and > 0");
    if (integrator != SD_EULER && integrator != SD_AB2) return fail(SD_EINVAL, "unknown integrator");
    if (steps < 0 || step0 < 0) return fail(SD_EINVAL, "steps and step0 must be >= 0");
    if (steps == 0) return SD_OK;
    hipStream_t hs = (hipStream_t)stream;
    const bool f64 = precision == SD_FP64;
    const size_t rec = f64 ? 32 : 16;
    const PairLaunch L = plan_pair(precision, n);
    void *partial = nullptr, *stage = nullptr, *F4 = nullptr;
    if ((st = ws_get(WS_PARTIAL, partial_bytes(L, n), &partial)) ||
        (st = ws_get(WS_STAGE, rec * (size_t)n, &stage)) ||
        (st = ws_get(WS_LUB_F, rec * (size_t)n, &F4)))
        return st;
    const double mu0 = 1.0 / (6.0 * M_PI * p->eta * p->a);
    // per step: forces with the correction (written straight into the force
    // records of the pair kernel), pair kernel, then merge + integrate, which
    // also stages the new positions for the next step
    hipError_t e = f64 ? launch_stage_f64(x, (double4*)stage, (int)n, hs)
                       : launch_stage_f32(x, (float4*)stage, (int)n, box_side(p), hs);
    if (e != hipSuccess) return fail(SD_EDEVICE, "staging launch: %s", hipGetErrorString(e));
    for (int64_t s = 0; s < steps; ++s) {
        const int64_t k = step0 + s;
        if ((st = lub_forces_impl(p, lub, n, x, v_prev, f_ext, nullptr,
                                  f64 ? nullptr : (float4*)F4, f64 ? (double4*)F4 : nullptr, hs)))
            return st;
        if ((st = run_pair(p, n, stage, F4, f64 ? nullptr : x, precision, (double*)partial, L, hs)))
            return st;
        // Euler: x += dt v, v_prev = v;  AB2: x += dt (3/2 v - 1/2 v_prev), v_prev = v
        const int mode = (integrator == SD_EULER) ? 0 : (k == 0 ? 1 : 2);
        const bool next = s + 1 < steps;
        e = f64 ? launch_merge_integrate_f64((double*)partial, L.splits, (int)n, (const double4*)F4,
                                             mu0, x, mode ? v_prev : nullptr,
                                             mode ? nullptr : v_prev, dt, mode,
                                             next ? (double4*)stage : nullptr, hs)
                : launch_merge_integrate_f32((double*)partial, L.splits, (int)n, (const float4*)F4,
                                             mu0, x, mode ? v_prev : nullptr,
                                             mode ? nullptr : v_prev, dt, mode,
                                             next ? (float4*)stage : nullptr, box_side(p), hs);
        if (e != hipSuccess) return fail(SD_EDEVICE, "integrate launch: %s", hipGetErrorString(e));
    }
    return SD_OK;
}

}  // extern "C"
