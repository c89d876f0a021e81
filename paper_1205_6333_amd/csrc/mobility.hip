// mobility.hip -- all-pairs mobility product v_i = mu0 F_i + sum_{j != i} T(r_i - r_j) F_j
// (Eq. 7a; tensors of Eq. 4 and Eq. 7b), hand-written for gfx950.
//
// Work decomposition: one lane owns one (or ILP) particle(s) i and walks a
// contiguous j-range; the j-range of all N particles is cut into `splits`
// chunks so that N = 65536 still puts several waves on every SIMD.  Each
// (i, split) writes one FP64 partial per component; a merge kernel adds the
// self term mu0 F_i and the partials in a fixed order (deterministic, no
// atomics).
//
// Precision: the far-field pair term is evaluated in FP32 (v_rsq_f32 on the
// VALU) and accumulated with Kahan compensation in FP32; pairs with
// r^2 < (2a)^2 (1 + NEAR_EPS), the self pair and coincident spheres are
// evaluated in FP64 on a rarely taken branch.  SD_FP64 runs the same loop in
// double.
#include "pair_terms.h"
#include "sd_internal.h"
#include "sym_chunk_asm.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace sd {

PairConst make_pair_const(double a, double eta, int tensor, int overlap, double box)
{
    PairConst c;
    const double gamma = (tensor == T_RPY) ? 2.0 * a * a / 3.0 : 0.0;
    const double thr2 = 4.0 * a * a * (1.0 + NEAR_EPS);
    // FP32 length unit: 1 in free space, the fixed-point unit s in a box
    const double s = box > 0.0 ? box / 4294967296.0 : 1.0;
    c.gamma_f = (float)(gamma / (s * s));
    c.m3gamma_f = (float)(-3.0 * gamma / (s * s));
    c.thr2_f = (float)(thr2 / (s * s));
    c.overlap = (tensor == T_RPY && overlap) ? 1 : 0;
    c.thr2_d = thr2;
    c.alpha = 1.0 / (8.0 * M_PI * eta);
    c.alpha_sum = c.alpha / s;
    c.gamma = gamma;
    c.mu0 = 1.0 / (6.0 * M_PI * eta * a);
    c.a = a;
    c.box = box > 0.0 ? box : 0.0;
    c.ibox = box > 0.0 ? 1.0 / box : 0.0;
    c.s_q = box > 0.0 ? s : 0.0;
    return c;
}

PairLaunch shape_pair_launch(int n, int variant, int block, int splits, int ilp, int cus)
{
    PairLaunch L;
    L.variant = variant;
    L.block = block;
    L.ilp = ilp;
    L.acc = 0;
    L.cus = 0;
    if (variant == 2) {
        // rows: the symmetric splits, the diagonal blocks, the folded j side
        L.jchunk = splits < 1 ? 1 : splits;
        L.cus = cus;
        const SymShape sh = sym_shape(n, block * ilp, L.jchunk, sym_slots(block, cus));
        L.splits = sh.isplits + 2;
        return L;
    }
    if (splits < 1) splits = 1;
    // j chunks are whole tiles of `block` particles
    const int tiles = (n + block - 1) / block;
    if (splits > tiles) splits = tiles;
    const int tiles_per = (tiles + splits - 1) / splits;
    L.jchunk = tiles_per * block;
    L.splits = (n + L.jchunk - 1) / L.jchunk;
    return L;
}

// Work-group -> (i-block, j-split).  Work-groups are dispatched round-robin
// over the 8 XCDs (linear id L runs on XCD L mod 8), each with its own L2.
// When the split count is a multiple of 8, split s is only ever handled by
// XCD s mod 8, so every XCD streams 1/8 of the j data through its L2.
__device__ __forceinline__ void map_block(int S, int& ib, int& s)
{
    const int L = blockIdx.x;
    if ((S & 7) == 0) {
        const int per = S >> 3;
        const int r = L >> 3;
        s = (r % per) * 8 + (L & 7);
        ib = r / per;
    } else {
        s = L % S;
        ib = L / S;
    }
}

// Placeholders for padded lanes / padded tile slots.  Far apart, zero force:
// every term they produce is exactly zero or never stored, and never NaN.
// In a periodic box no point is far from another; there the placeholders are
// the origin, and a placeholder that lands below the near threshold takes the
// near branch, which skips padded indices and masks the pair to +inf.
#define SD_FAR_I (-1.0e15f)
#define SD_FAR_J (1.0e15f)

template <bool PER>
__device__ __forceinline__ float far_i() { return PER ? 0.0f : SD_FAR_I; }
template <bool PER>
__device__ __forceinline__ float far_j() { return PER ? 0.0f : SD_FAR_J; }

// FP32 coordinate difference a - b.  Periodic: a and b hold fixed-point bits;
// the 32-bit wrapped difference is the nearest image in units of s.
template <bool PER>
__device__ __forceinline__ float pdiff(float a, float b)
{
    if (PER) return (float)(int)(__float_as_uint(a) - __float_as_uint(b));
    return a - b;
}

// FP32 constants of the pair terms, held in VGPRs.  On gfx950 a VALU
// instruction that reads an SGPR operand issues at half the rate of one that
// reads VGPRs only (measured: 4.1 vs 2.2 cycles per wave instruction and
// SIMD), and the compiler keeps wave-uniform values in SGPRs; the empty asm
// makes the values lane values.  `one` keeps the literal 1.0 out of the
// coefficient's FMA for the same reason.
struct VConst {
    float gamma, m3g, thr2, one;
};

__device__ __forceinline__ VConst vconst(const PairConst& pc)
{
    VConst k{pc.gamma_f, pc.m3gamma_f, pc.thr2_f, 1.0f};
    asm volatile("" : "+v"(k.gamma), "+v"(k.m3g), "+v"(k.thr2), "+v"(k.one));
    return k;
}

// Per-lane state of one particle i.
struct LaneF32 {
    float x, y, z;        // position (FP32)
    float s0, s1, s2;     // running sums (scaled units)
    float c0, c1, c2;     // Kahan compensations
    double n0, n1, n2;    // FP64 near-pair sums (physical units)
    int i;
};

// FP64 difference x_i - x_j of a near pair: from the FP64 positions when
// given (nearest image in a box), else from the FP32 records (exact
// difference of floats, or the fixed-point difference times s).
template <bool PER>
__device__ __forceinline__ void near_diff(const LaneF32& L, const float4 pj, int jg,
                                          const PairConst& pc, const double* __restrict__ x64,
                                          double& d0, double& d1, double& d2)
{
    if (x64) {
        d0 = x64[3 * (size_t)L.i + 0] - x64[3 * (size_t)jg + 0];
        d1 = x64[3 * (size_t)L.i + 1] - x64[3 * (size_t)jg + 1];
        d2 = x64[3 * (size_t)L.i + 2] - x64[3 * (size_t)jg + 2];
        if (PER) nearest_image_d(pc, d0, d1, d2);
    } else if (PER) {
        d0 = (double)(int)(__float_as_uint(L.x) - __float_as_uint(pj.x)) * pc.s_q;
        d1 = (double)(int)(__float_as_uint(L.y) - __float_as_uint(pj.y)) * pc.s_q;
        d2 = (double)(int)(__float_as_uint(L.z) - __float_as_uint(pj.z)) * pc.s_q;
    } else {
        d0 = (double)L.x - (double)pj.x;
        d1 = (double)L.y - (double)pj.y;
        d2 = (double)L.z - (double)pj.z;
    }
}

// Unordered pairs i < j met by the product kernels on this device that break
// the premise r >= 2a of Eq. 4: [0] with 0 < r < 2a, [1] with r = 0.  Counted
// on the rare FP64 near-pair branch only, by the evaluation of row min(i, j).
__device__ unsigned long long g_premise[2];

// Called by the lanes active at that point, each with the class of its pair
// (PREMISE_OK for none): one atomic add per class and call, by one lane, for
// the whole wave (a dense suspension meets thousands of such pairs per
// product, and atomics on one address serialise).
__device__ __forceinline__ void count_premise(int cls)
{
    const uint64_t sub = __builtin_amdgcn_ballot_w64(cls == PREMISE_SUB2A);
    const uint64_t co = __builtin_amdgcn_ballot_w64(cls == PREMISE_COINCIDENT);
    if ((sub | co) == 0) return;
    const uint64_t act = __builtin_amdgcn_ballot_w64(true);
    if ((int)(threadIdx.x & 63) != __builtin_ctzll(act)) return;
    if (sub) atomicAdd(&g_premise[0], (unsigned long long)__builtin_popcountll(sub));
    if (co) atomicAdd(&g_premise[1], (unsigned long long)__builtin_popcountll(co));
}

// Per-lane counts, added for the wave with one atomic add per class (all
// lanes of the wave call it).
__device__ __forceinline__ void count_premise_lanes(uint32_t sub, uint32_t co)
{
    for (int off = 32; off > 0; off >>= 1) {
        sub += __shfl_xor(sub, off);
        co += __shfl_xor(co, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (sub) atomicAdd(&g_premise[0], (unsigned long long)sub);
        if (co) atomicAdd(&g_premise[1], (unsigned long long)co);
    }
}

// One pair (i, j) on the FP32 fast path.  pj/fj: position and force of j
// (wave-uniform).  jg: global index of j, used only on the near branch.
template <int TENSOR, bool KAHAN, bool PER>
__device__ __forceinline__ void pair_f32(LaneF32& L, const float4 pj, const float4 fj, int jg,
                                         int n, const PairConst& pc, float gamma, float m3g,
                                         float thr2, const double* __restrict__ x64)
{
    const float dx = pdiff<PER>(L.x, pj.x);
    const float dy = pdiff<PER>(L.y, pj.y);
    const float dz = pdiff<PER>(L.z, pj.z);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const bool nr = r2 < thr2;
    float rinv = __builtin_amdgcn_rsqf(r2);
    rinv = nr ? 0.0f : rinv;
    const float rinv2 = rinv * rinv;
    const float rinv3 = rinv2 * rinv;
    float A, Bt;
    if (TENSOR == T_OSEEN) {
        A = rinv;
        Bt = rinv3;
    } else {
        A = fmaf(gamma, rinv3, rinv);
        Bt = rinv3 * fmaf(m3g, rinv2, 1.0f);
    }
    const float dF = fmaf(dx, fj.x, fmaf(dy, fj.y, dz * fj.z));
    const float sB = Bt * dF;
    if (KAHAN) {
        // y = term - c, t = s + y, c = (t - s) - y, s = t
        const float y0 = fmaf(A, fj.x, fmaf(sB, dx, -L.c0));
        const float y1 = fmaf(A, fj.y, fmaf(sB, dy, -L.c1));
        const float y2 = fmaf(A, fj.z, fmaf(sB, dz, -L.c2));
        const float t0 = L.s0 + y0;
        const float t1 = L.s1 + y1;
        const float t2 = L.s2 + y2;
        L.c0 = (t0 - L.s0) - y0;
        L.c1 = (t1 - L.s1) - y1;
        L.c2 = (t2 - L.s2) - y2;
        L.s0 = t0;
        L.s1 = t1;
        L.s2 = t2;
    } else {
        L.s0 = fmaf(A, fj.x, fmaf(sB, dx, L.s0));
        L.s1 = fmaf(A, fj.y, fmaf(sB, dy, L.s1));
        L.s2 = fmaf(A, fj.z, fmaf(sB, dz, L.s2));
    }
    // padded lanes (i >= n) and padded tile slots (j >= n) never reach the FP64
    // evaluation: their placeholders are far from every particle, and the
    // index test below keeps x64 reads in bounds even for absurd inputs
    if (nr) {
        if (jg != L.i && L.i < n && jg < n) {
            double d0, d1, d2;
            near_diff<PER>(L, pj, jg, pc, x64, d0, d1, d2);
            const int cls = near_term<TENSOR>(pc, d0, d1, d2, (double)fj.x, (double)fj.y,
                                              (double)fj.z, L.n0, L.n1, L.n2);
            count_premise(L.i < jg ? cls : PREMISE_OK);
        }
    }
}

// FP64 evaluation of one near pair (r^2 below the threshold) of lane particle
// i, accumulated into the lane's own LDS slot (only the owning lane ever
// touches it, so no synchronisation is needed and the order is fixed).  The
// self pair and padded slots contribute nothing.
template <int TENSOR, bool PER>
__device__ __forceinline__ void near_pair_lds(const LaneF32& L, const float4 pj, const float4 fj,
                                           int jg, int n, const PairConst& pc,
                                           const double* __restrict__ x64, double* slot, int stride)
{
    if (jg == L.i || L.i >= n || jg >= n) return;
    double d0, d1, d2;
    near_diff<PER>(L, pj, jg, pc, x64, d0, d1, d2);
    double n0 = slot[0], n1 = slot[stride], n2 = slot[2 * stride];
    const int cls =
        near_term<TENSOR>(pc, d0, d1, d2, (double)fj.x, (double)fj.y, (double)fj.z, n0, n1, n2);
    count_premise(L.i < jg ? cls : PREMISE_OK);
    slot[0] = n0;
    slot[stride] = n1;
    slot[2 * stride] = n2;
}

// A group of U pairs (i, j_0..j_{U-1}) for every lane particle.  The near test
// is done once per group: only if some lane of the wave has a pair below the
// threshold does the group take the rare branch, which evaluates those pairs
// in FP64 (near_pair_lds) and sets their r^2 to +inf, so that the FP32 code
// below gives them rinv = 0 and an exact zero contribution.  The FP32 code is
// the same for every group.
// ACC: 0 = plain FP32 sums, k >= 1 = Kahan compensation applied once per k
// consecutive terms (k = 1: per term).
template <int TENSOR, int ACC, int U, int ILP, bool PER>
__device__ __forceinline__ void pair_group(LaneF32 (&L)[ILP], const float4 (&pj)[U],
                                           const float4 (&fj)[U], int jg0, int n,
                                           const PairConst& pc, const VConst& kc,
                                           const double* __restrict__ x64, double* near_slot,
                                           int stride)
{
    const float gamma = kc.gamma, m3g = kc.m3g, thr2 = kc.thr2;
    float dx[ILP][U], dy[ILP][U], dz[ILP][U], r2[ILP][U];
    float rmin = 0.0f;
#pragma unroll
    for (int q = 0; q < ILP; ++q)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dx[q][u] = pdiff<PER>(L[q].x, pj[u].x);
            dy[q][u] = pdiff<PER>(L[q].y, pj[u].y);
            dz[q][u] = pdiff<PER>(L[q].z, pj[u].z);
            r2[q][u] = fmaf(dx[q][u], dx[q][u], fmaf(dy[q][u], dy[q][u], dz[q][u] * dz[q][u]));
            rmin = (q == 0 && u == 0) ? r2[q][u] : fminf(rmin, r2[q][u]);
        }
    if (__builtin_amdgcn_ballot_w64(rmin < thr2) != 0) {
#pragma unroll
        for (int q = 0; q < ILP; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (r2[q][u] < thr2)
                    near_pair_lds<TENSOR, PER>(L[q], pj[u], fj[u], jg0 + u, n, pc, x64,
                                          near_slot + q * (stride / ILP), stride);
                r2[q][u] = (r2[q][u] < thr2) ? __builtin_inff() : r2[q][u];
            }
    }
#pragma unroll
    for (int q = 0; q < ILP; ++q) {
        constexpr int KB = ACC > 0 ? ACC : 1;
#pragma unroll
        for (int u0 = 0; u0 < U; u0 += KB) {
            float y0 = ACC ? -L[q].c0 : L[q].s0;
            float y1 = ACC ? -L[q].c1 : L[q].s1;
            float y2 = ACC ? -L[q].c2 : L[q].s2;
#pragma unroll
            for (int u = u0; u < u0 + KB; ++u) {
                const float rinv = __builtin_amdgcn_rsqf(r2[q][u]);
                const float rinv2 = rinv * rinv;
                const float rinv3 = rinv2 * rinv;
                float A, Bt;
                if (TENSOR == T_OSEEN) {
                    A = rinv;
                    Bt = rinv3;
                } else {
                    A = fmaf(gamma, rinv3, rinv);
                    Bt = rinv3 * fmaf(m3g, rinv2, kc.one);
                }
                const float dF = fmaf(dx[q][u], fj[u].x, fmaf(dy[q][u], fj[u].y, dz[q][u] * fj[u].z));
                const float sB = Bt * dF;
                y0 = fmaf(A, fj[u].x, fmaf(sB, dx[q][u], y0));
                y1 = fmaf(A, fj[u].y, fmaf(sB, dy[q][u], y1));
                y2 = fmaf(A, fj[u].z, fmaf(sB, dz[q][u], y2));
            }
            if (ACC) {
                const float t0 = L[q].s0 + y0;
                const float t1 = L[q].s1 + y1;
                const float t2 = L[q].s2 + y2;
                L[q].c0 = (t0 - L[q].s0) - y0;
                L[q].c1 = (t1 - L[q].s1) - y1;
                L[q].c2 = (t2 - L[q].s2) - y2;
                L[q].s0 = t0;
                L[q].s1 = t1;
                L[q].s2 = t2;
            } else {
                L[q].s0 = y0;
                L[q].s1 = y1;
                L[q].s2 = y2;
            }
        }
    }
}

template <int ILP, int BLOCK, bool PER>
__device__ __forceinline__ void lanes_init(LaneF32 (&L)[ILP], const float4* __restrict__ pos, int n,
                                           int ib)
{
    const int ibase = ib * (BLOCK * ILP) + threadIdx.x;
#pragma unroll
    for (int q = 0; q < ILP; ++q) {
        const int i = ibase + q * BLOCK;
        L[q].i = i;
        if (i < n) {
            const float4 p = pos[i];
            L[q].x = p.x;
            L[q].y = p.y;
            L[q].z = p.z;
        } else {
            L[q].x = L[q].y = L[q].z = far_i<PER>();
        }
        L[q].s0 = L[q].s1 = L[q].s2 = 0.0f;
        L[q].c0 = L[q].c1 = L[q].c2 = 0.0f;
        L[q].n0 = L[q].n1 = L[q].n2 = 0.0;
    }
}

// near_slot: this lane's LDS near-pair sums (component k of particle q at
// near_slot[k * stride + q * stride / ILP]).
template <int ILP>
__device__ __forceinline__ void lanes_store(const LaneF32 (&L)[ILP], int n, int s, double alpha,
                                            const double* near_slot, int stride,
                                            double* __restrict__ partial)
{
#pragma unroll
    for (int q = 0; q < ILP; ++q) {
        const int i = L[q].i;
        const double* ns = near_slot + q * (stride / ILP);
        if (i < n) {
            const size_t base = (size_t)s * 3 * (size_t)n + (size_t)i;
            partial[base] = alpha * ((double)L[q].s0 - (double)L[q].c0) + (L[q].n0 + ns[0]);
            partial[base + (size_t)n] =
                alpha * ((double)L[q].s1 - (double)L[q].c1) + (L[q].n1 + ns[stride]);
            partial[base + 2 * (size_t)n] =
                alpha * ((double)L[q].s2 - (double)L[q].c2) + (L[q].n2 + ns[2 * stride]);
        }
    }
}

template <int ILP, int BLOCK>
__device__ __forceinline__ double* near_slots_init(double* s_near)
{
    double* slot = s_near + threadIdx.x;
#pragma unroll
    for (int k = 0; k < 3 * ILP; ++k) slot[k * BLOCK] = 0.0;
    return slot;
}

// pairs per near test; a Kahan block of 8 terms uses groups of 8
template <int ACC>
struct GroupSize {
    static constexpr int value = ACC > 4 ? ACC : 4;
};

// Variant 0: the work-group stages tiles of BLOCK j-particles (position and
// force, 32 B each) in LDS with coalesced 16-byte loads; the next tile is
// fetched into registers while the current one is consumed.  Every lane then
// reads each j from LDS by broadcast.
template <int TENSOR, int ACC, int BLOCK, int ILP, bool PER>
__global__ void __launch_bounds__(BLOCK)
k_pair_f32_lds(const float4* __restrict__ pos, const float4* __restrict__ frc,
               const double* __restrict__ x64, int n, int jchunk, int S, PairConst pc,
               double* __restrict__ partial)
{
    __shared__ float4 s_pos[BLOCK];
    __shared__ float4 s_frc[BLOCK];
    __shared__ double s_near[3 * BLOCK * ILP];
    int ib, s;
    map_block(S, ib, s);
    LaneF32 L[ILP];
    lanes_init<ILP, BLOCK, PER>(L, pos, n, ib);
    double* near_slot = near_slots_init<ILP, BLOCK>(s_near);
    constexpr int NS = BLOCK * ILP;
    constexpr int GROUP_U = GroupSize<ACC>::value;
    const int tid = threadIdx.x;
    const int jbeg = s * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const VConst kc = vconst(pc);
    const float4 far_j4 = make_float4(far_j<PER>(), far_j<PER>(), far_j<PER>(), 0.0f);
    const float4 zero4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);

    float4 rp = far_j4, rf = zero4;
    if (jbeg + tid < jend) {
        rp = pos[jbeg + tid];
        rf = frc[jbeg + tid];
    }
    for (int jt = jbeg; jt < jend; jt += BLOCK) {
        __syncthreads();
        s_pos[tid] = rp;
        s_frc[tid] = rf;
        __syncthreads();
        const int jn = jt + BLOCK + tid;
        rp = far_j4;
        rf = zero4;
        if (jn < jend) {
            rp = pos[jn];
            rf = frc[jn];
        }
        for (int k = 0; k < BLOCK; k += GROUP_U) {
            float4 pj[GROUP_U], fj[GROUP_U];
#pragma unroll
            for (int u = 0; u < GROUP_U; ++u) {
                pj[u] = s_pos[k + u];
                fj[u] = s_frc[k + u];
            }
            pair_group<TENSOR, ACC, GROUP_U, ILP, PER>(L, pj, fj, jt + k, n, pc, kc, x64,
                                                       near_slot, NS);
        }
    }
    lanes_store<ILP>(L, n, s, pc.alpha_sum, near_slot, NS, partial);
}

// Variant 1: no LDS.  The j index is wave-uniform, so positions and forces of
// j are fetched with scalar loads through the scalar cache (the paper's
// "naive" cache-based read of Sec. 3.2, on AMD's scalar path) and enter the
// VALU as SGPR operands.
template <int TENSOR, int ACC, int BLOCK, int ILP, bool PER>
__global__ void __launch_bounds__(BLOCK)
k_pair_f32_smem(const float4* __restrict__ pos, const float4* __restrict__ frc,
                const double* __restrict__ x64, int n, int jchunk, int S, PairConst pc,
                double* __restrict__ partial)
{
    __shared__ double s_near[3 * BLOCK * ILP];
    int ib, s;
    map_block(S, ib, s);
    LaneF32 L[ILP];
    lanes_init<ILP, BLOCK, PER>(L, pos, n, ib);
    double* near_slot = near_slots_init<ILP, BLOCK>(s_near);
    constexpr int NS = BLOCK * ILP;
    constexpr int GROUP_U = GroupSize<ACC>::value;
    const int jbeg = s * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const float gamma = pc.gamma_f, m3g = pc.m3gamma_f, thr2 = pc.thr2_f;
    const VConst kc = vconst(pc);
    int j = jbeg;
    for (; j + GROUP_U <= jend; j += GROUP_U) {
        float4 pj[GROUP_U], fj[GROUP_U];
#pragma unroll
        for (int u = 0; u < GROUP_U; ++u) {
            pj[u] = pos[j + u];
            fj[u] = frc[j + u];
        }
        pair_group<TENSOR, ACC, GROUP_U, ILP, PER>(L, pj, fj, j, n, pc, kc, x64, near_slot,
                                                   NS);
    }
    for (; j < jend; ++j) {
        const float4 pj = pos[j];
        const float4 fj = frc[j];
#pragma unroll
        for (int q = 0; q < ILP; ++q)
            pair_f32<TENSOR, ACC != 0, PER>(L[q], pj, fj, j, n, pc, gamma, m3g, thr2, x64);
    }
    lanes_store<ILP>(L, n, s, pc.alpha_sum, near_slot, NS, partial);
}

// ------------------------------------------------ variant 2: pair symmetry
//
// The blocks of M satisfy M_ji = M_ij^T and T is even in r (Sec. 3.3 uses
// mu_ij = mu_ji on the CPU), so one evaluation of the coefficients A', Bt' of
// a pair gives both T(r_ij) F_j for i and T(r_ij) F_i for j.  Variant 2
// evaluates every pair of particles in different blocks once:
//
// Block schedule.  Particles are cut into nb blocks of B = BLOCK * ILP
// (ILP particles per lane, see k_pair_f32_sym).  Work-group
// (I, s) owns i-block I.  The blocks J = I + 1 .. I + h (mod nb), h =
// (nb - 1) / 2, and, when nb is even, J = I + nb/2 for I < nb/2 only, form a
// virtual j range p = (J - I - 1 mod nb) B + offset, cut into splits of
// `chunk` positions.  Every unordered pair of distinct blocks is thus taken
// exactly once.  The diagonal blocks J = I are taken one-sided (every ordered
// pair, as variant 0) by nb extra work-groups dispatched last.
//
// Rows of 16 lanes.  Each 16-lane row of a wave holds 16 (ILP 2: 32)
// particles i, one (two) per lane.  A tile of SYM_TJ particles j is staged in
// LDS in chunks of 16, each chunk stored twice in a row, so that lane q reads
// element (q + k) mod 16 of a chunk at the constant offset k.  In step k of a
// chunk lane q pairs its i with that element; the j-side term goes to the
// lane that owns the element through a DPP row rotation (row_ror:k: lane m
// reads lane m - k), so every lane accumulates the j-side sum of one element
// of the chunk (16 steps, at most 32 terms, in FP32) and no cross-lane
// reduction is needed.  After a chunk each row stores its 16 j-side sums in
// LDS; at the end of a tile the rows are added in FP64 in a fixed order and
// written as FP32 j-side partials jpart[c][I][p] (scaled units), which
// k_sym_fold_near adds in FP64, in a fixed order, into one more split row
// (or, for a product, straight into the merged velocities).
// Tiles are double-buffered: the next tile is read from HBM while the
// current one is consumed, so a tile costs two barriers.
//
// Near pairs.  A pair with r^2 below the near threshold (near contact,
// overlap, coincident spheres) contributes nothing here, on either side: its
// r^2 is replaced by +inf, so that rsq gives 0.  The wave records instead,
// in a flag matrix over runs of SYM_RUN = 64 consecutive particles, every
// pair of runs that holds one of its particles and one particle of the tile,
// and k_sym_fold_near evaluates every pair of the flagged run pairs in FP64,
// one-sided (both orderings), with the same FP32 threshold test, so that
// exactly the masked pairs are added back.  The hot loop thus holds no FP64
// code and no function call, and a near pair costs the fold 64 x 64 distance
// tests, not a whole block pair.

// Split schedule.  The i-blocks' virtual j ranges are cut alike, and the
// launch orders its work-groups diagonal blocks first, then split 0 of every
// i-block, split 1, ...  The hardware starts work-groups in that order as
// resident ones finish, so the work-groups that run last are the short ones:
// a split takes about the share of the remaining range that one round of
// resident work-groups covers (nb * size / slots of it, at most 1/splits of
// the whole range, at least one tile), which leaves a tail of about one tile
// instead of one whole split.
SymShape sym_shape(int n, int block, int splits, int slots)
{
    SymShape sh;
    sh.nb = (n + block - 1) / block;
    sh.h = (sh.nb - 1) / 2;
    sh.extra = (sh.nb >= 2 && (sh.nb & 1) == 0) ? 1 : 0;
    sh.lmax = (sh.h + sh.extra) * block;
    sh.nt = sh.lmax / SYM_TJ;
    const int tiles = sh.lmax / SYM_TJ;
    const int sp = splits < 1 ? 1 : splits;
    const int64_t big = std::max<int64_t>(1, (tiles + sp - 1) / sp);
    const int64_t sl = std::max(1, slots);
    int k = 0, at = 0;
    sh.off[0] = 0;
    while (at < tiles) {
        const int64_t left = tiles - at;
        int64_t size = (left * sh.nb + sl - 1) / sl;
        size = std::min(std::max<int64_t>(size, 1), big);
        if (k == SYM_MAX_SPLITS - 1) size = left;
        at += (int)std::min(size, left);
        sh.off[++k] = at;
    }
    if (k == 0) sh.off[++k] = 0;   // one empty split (a single block)
    sh.isplits = k;
    for (int m = k + 1; m <= SYM_MAX_SPLITS; ++m) sh.off[m] = at;
    return sh;
}

int sym_slots(int block, int cus)
{
    // LDS per work-group (two staged tiles or one block, the j-side rows)
    // against 160 KiB per CU, and at most 16 resident waves per CU (four per
    // SIMD: the register budget of the kernel)
    const int lds = 2 * 512 * 16 + 3 * (block / 16) * SYM_TJ * 4;
    const int by_lds = (160 * 1024) / lds;
    const int by_waves = 16 / (block / 64) > 0 ? 16 / (block / 64) : 1;
    return std::max(1, std::min(by_lds, by_waves)) * std::max(1, cus);
}

SymShape sym_shape_of(const PairLaunch& L, int n)
{
    return sym_shape(n, L.block * L.ilp, L.jchunk, sym_slots(L.block, L.cus));
}

size_t sym_flags_bytes(const SymShape& sh, int block)
{
    const size_t rows = (size_t)sh.nb * (size_t)(block / SYM_RUN);
    return (rows * (size_t)sh.nt + rows) * sizeof(uint4);
}

size_t sym_jpart_floats(const SymShape& sh) { return (size_t)3 * sh.nb * (size_t)sh.lmax; }

size_t sym_jpart_offset(const PairLaunch& L, int64_t n)
{
    const size_t b = (size_t)L.splits * 3 * (size_t)n * sizeof(double);
    return (b + 255) & ~(size_t)255;
}

size_t sym_flags_offset(const PairLaunch& L, int64_t n)
{
    const size_t b = sym_jpart_offset(L, n) +
                     sym_jpart_floats(sym_shape_of(L, (int)n)) * sizeof(float);
    return (b + 255) & ~(size_t)255;
}

size_t sym_workspace_bytes(const PairLaunch& L, int64_t n)
{
    return sym_flags_offset(L, n) + sym_flags_bytes(sym_shape_of(L, (int)n), L.block * L.ilp);
}

// Compile-time loop: f(integral_constant<int, U>) for U = B .. E-1.
template <int B, int E>
struct StaticFor {
    template <class F>
    __device__ __forceinline__ static void run(F&& f)
    {
        f(std::integral_constant<int, B>());
        StaticFor<B + 1, E>::run(f);
    }
};
template <int E>
struct StaticFor<E, E> {
    template <class F>
    __device__ __forceinline__ static void run(F&&) {}
};

// acc + (value v of lane (lane - K) mod 16 of the same row)
template <int K>
__device__ __forceinline__ float add_row_rot(float acc, float v)
{
    if constexpr (K == 0) {
        return acc + v;
    } else {
        return acc + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                                  0, __builtin_bit_cast(int, v), 0x120 + K, 0xf,
                                                  0xf, true));
    }
}

// Per-lane state of one particle i of the symmetric kernel (FP32 only).
struct SymLane {
    float x, y, z;        // position
    float s0, s1, s2;     // running sums of the i side (scaled units)
    float c0, c1, c2;     // Kahan compensations
};

template <int ILP, int BLOCK, bool PER>
__device__ __forceinline__ void sym_lanes_init(SymLane (&L)[ILP], const float4* __restrict__ pos,
                                               int n, int ib)
{
    const int ibase = ib * (BLOCK * ILP) + (int)threadIdx.x;
#pragma unroll
    for (int l = 0; l < ILP; ++l) {
        const int i = ibase + l * BLOCK;
        if (i < n) {
            const float4 p = pos[i];
            L[l].x = p.x;
            L[l].y = p.y;
            L[l].z = p.z;
        } else {
            L[l].x = L[l].y = L[l].z = far_i<PER>();
        }
        L[l].s0 = L[l].s1 = L[l].s2 = 0.0f;
        L[l].c0 = L[l].c1 = L[l].c2 = 0.0f;
    }
}

// i-side sums of the lane particles -> split row s (FP64, physical units)
template <int ILP, int BLOCK>
__device__ __forceinline__ void sym_lanes_store(const SymLane (&L)[ILP], int n, int ib, int s,
                                                double alpha, double* __restrict__ partial)
{
    const int ibase = ib * (BLOCK * ILP) + (int)threadIdx.x;
#pragma unroll
    for (int l = 0; l < ILP; ++l) {
        const int i = ibase + l * BLOCK;
        if (i < n) {
            const size_t base = (size_t)s * 3 * (size_t)n + (size_t)i;
            partial[base] = alpha * ((double)L[l].s0 - (double)L[l].c0);
            partial[base + (size_t)n] = alpha * ((double)L[l].s1 - (double)L[l].c1);
            partial[base + 2 * (size_t)n] = alpha * ((double)L[l].s2 - (double)L[l].c2);
        }
    }
}

// Steps K0 .. K0+U-1 of a chunk for one lane and its ILP particles i: pairs
// (i, element (q + k) mod 16).  sp/sf: this lane's view of the doubled chunk
// (element (q + k) mod 16 at offset k).  y: the running FP32 sums of the i
// side (for ACC > 0 the terms since the last compensated add, started from
// -c; for ACC = 0 the sums themselves); a compensation block of ACC terms may
// span groups.  aj*: the j-side sums of element q (scaled units), started by
// step 0.  near: set when a pair of the group is below the near threshold
// (that pair then contributes nothing).
template <int TENSOR, int ACC, bool PER, int K0, int U, int ILP>
__device__ __forceinline__ void sym_steps(SymLane (&L)[ILP], const float (&fi)[ILP][3],
                                          float (&y)[ILP][3], float& aj0, float& aj1, float& aj2,
                                          const float4* sp, const float4* sf,
                                          const VConst& kc, uint64_t& near)
{
    const float gamma = kc.gamma, m3g = kc.m3g, thr2 = kc.thr2;
    constexpr int KB = ACC > 0 ? ACC : 1;
    static_assert(ACC == 0 || KB % U == 0 || U % KB == 0, "compensation blocks and groups");
    // groups are scheduled one after the other: overlapping them would hold
    // two groups of pair data in registers
    __builtin_amdgcn_sched_barrier(0);
    float pjx[U], pjy[U], pjz[U], fjx[U], fjy[U], fjz[U];
    float dx[ILP][U], dy[ILP][U], dz[ILP][U], r2[ILP][U];
    float rmin = 0.0f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const float4 p = sp[K0 + u];
        const float4 f = sf[K0 + u];
        pjx[u] = p.x;
        pjy[u] = p.y;
        pjz[u] = p.z;
        fjx[u] = f.x;
        fjy[u] = f.y;
        fjz[u] = f.z;
#pragma unroll
        for (int l = 0; l < ILP; ++l) {
            dx[l][u] = pdiff<PER>(L[l].x, pjx[u]);
            dy[l][u] = pdiff<PER>(L[l].y, pjy[u]);
            dz[l][u] = pdiff<PER>(L[l].z, pjz[u]);
            r2[l][u] = fmaf(dx[l][u], dx[l][u], fmaf(dy[l][u], dy[l][u], dz[l][u] * dz[l][u]));
            rmin = (l == 0 && u == 0) ? r2[l][u] : fminf(rmin, r2[l][u]);
        }
    }
    const uint64_t nearb = __builtin_amdgcn_ballot_w64(rmin < thr2);
    if (nearb != 0) {   // rare
        near |= nearb;
#pragma unroll
        for (int l = 0; l < ILP; ++l)
#pragma unroll
            for (int u = 0; u < U; ++u) r2[l][u] = (r2[l][u] < thr2) ? __builtin_inff() : r2[l][u];
    }
    StaticFor<0, U>::run([&](auto u_c) {
        constexpr int u = decltype(u_c)::value;
        constexpr int k = K0 + u;   // step within the chunk
        if constexpr (ACC == 0 ? u == 0 : k % KB == 0) {
#pragma unroll
            for (int l = 0; l < ILP; ++l) {
                y[l][0] = ACC ? -L[l].c0 : L[l].s0;
                y[l][1] = ACC ? -L[l].c1 : L[l].s1;
                y[l][2] = ACC ? -L[l].c2 : L[l].s2;
            }
        }
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
        for (int l = 0; l < ILP; ++l) {
            const float rinv = __builtin_amdgcn_rsqf(r2[l][u]);
            const float rinv2 = rinv * rinv;
            const float rinv3 = rinv2 * rinv;
            float A, Bt;
            if (TENSOR == T_OSEEN) {
                A = rinv;
                Bt = rinv3;
            } else {
                A = fmaf(gamma, rinv3, rinv);
                Bt = rinv3 * fmaf(m3g, rinv2, kc.one);
            }
            // i side: T F_j
            const float dFj = fmaf(dx[l][u], fjx[u], fmaf(dy[l][u], fjy[u], dz[l][u] * fjz[u]));
            const float sBj = Bt * dFj;
            y[l][0] = fmaf(A, fjx[u], fmaf(sBj, dx[l][u], y[l][0]));
            y[l][1] = fmaf(A, fjy[u], fmaf(sBj, dy[l][u], y[l][1]));
            y[l][2] = fmaf(A, fjz[u], fmaf(sBj, dz[l][u], y[l][2]));
            // j side: T F_i of this lane's particles, summed before the hand-over
            const float dFi =
                fmaf(dx[l][u], fi[l][0], fmaf(dy[l][u], fi[l][1], dz[l][u] * fi[l][2]));
            const float sBi = Bt * dFi;
            if (l == 0) {
                c0 = fmaf(A, fi[l][0], sBi * dx[l][u]);
                c1 = fmaf(A, fi[l][1], sBi * dy[l][u]);
                c2 = fmaf(A, fi[l][2], sBi * dz[l][u]);
            } else {
                c0 = fmaf(A, fi[l][0], fmaf(sBi, dx[l][u], c0));
                c1 = fmaf(A, fi[l][1], fmaf(sBi, dy[l][u], c1));
                c2 = fmaf(A, fi[l][2], fmaf(sBi, dz[l][u], c2));
            }
        }
        // hand the j-side term to the lane that owns the element
        if constexpr (k == 0) {   // the first step of a chunk starts the sums
            aj0 = c0;
            aj1 = c1;
            aj2 = c2;
        } else {
            aj0 = add_row_rot<k & 15>(aj0, c0);
            aj1 = add_row_rot<k & 15>(aj1, c1);
            aj2 = add_row_rot<k & 15>(aj2, c2);
        }
        if constexpr (ACC == 0 ? u == U - 1 : k % KB == KB - 1) {
#pragma unroll
            for (int l = 0; l < ILP; ++l) {
                if (ACC) {
                    // Fast2Sum: s + y exactly as t + (y - (t - s)), c = -(y - (t - s))
                    const float t0 = L[l].s0 + y[l][0];
                    const float t1 = L[l].s1 + y[l][1];
                    const float t2 = L[l].s2 + y[l][2];
                    L[l].c0 = (t0 - L[l].s0) - y[l][0];
                    L[l].c1 = (t1 - L[l].s1) - y[l][1];
                    L[l].c2 = (t2 - L[l].s2) - y[l][2];
                    L[l].s0 = t0;
                    L[l].s1 = t1;
                    L[l].s2 = t2;
                } else {
                    L[l].s0 = y[l][0];
                    L[l].s1 = y[l][1];
                    L[l].s2 = y[l][2];
                }
            }
        }
    });
    // The sums are materialised here: otherwise their addition chains are
    // sunk towards their only use at the end of the chunk, and the terms of
    // all steps stay live until then.
    asm volatile("" : "+v"(aj0), "+v"(aj1), "+v"(aj2));
#pragma unroll
    for (int l = 0; l < ILP; ++l)
        asm volatile("" : "+v"(y[l][0]), "+v"(y[l][1]), "+v"(y[l][2]), "+v"(L[l].s0),
                     "+v"(L[l].s1), "+v"(L[l].s2), "+v"(L[l].c0), "+v"(L[l].c1), "+v"(L[l].c2));
}

// Diagonal block, one-sided: a group of G particles j (broadcast LDS reads)
// for every lane particle.  ig: global indices of the lane particles, jg0:
// global index of the group's first j.  Near pairs are masked as in
// sym_steps; near is set only for pairs other than a particle with itself.
// ACC: 0 plain FP32 sums, k >= 1 Kahan compensation once per k terms.
template <int TENSOR, int ACC, int G, int ILP, bool PER>
__device__ __forceinline__ void diag_group(SymLane (&L)[ILP], const int (&ig)[ILP],
                                           const float4 (&pjv)[G], const float4 (&fjv)[G],
                                           int jg0, const VConst& kc, uint64_t& near)
{
    const float gamma = kc.gamma, m3g = kc.m3g, thr2 = kc.thr2;
    float pjx[G], pjy[G], pjz[G], fjx[G], fjy[G], fjz[G];
    float dx[ILP][G], dy[ILP][G], dz[ILP][G], r2[ILP][G];
    float rmin = 0.0f;
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const float4 p = pjv[u];
        const float4 f = fjv[u];
        pjx[u] = p.x;
        pjy[u] = p.y;
        pjz[u] = p.z;
        fjx[u] = f.x;
        fjy[u] = f.y;
        fjz[u] = f.z;
#pragma unroll
        for (int l = 0; l < ILP; ++l) {
            dx[l][u] = pdiff<PER>(L[l].x, pjx[u]);
            dy[l][u] = pdiff<PER>(L[l].y, pjy[u]);
            dz[l][u] = pdiff<PER>(L[l].z, pjz[u]);
            r2[l][u] = fmaf(dx[l][u], dx[l][u], fmaf(dy[l][u], dy[l][u], dz[l][u] * dz[l][u]));
            rmin = (l == 0 && u == 0) ? r2[l][u] : fminf(rmin, r2[l][u]);
        }
    }
    if (__builtin_amdgcn_ballot_w64(rmin < thr2) != 0) {
        bool other = false;
#pragma unroll
        for (int l = 0; l < ILP; ++l)
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const bool nr = r2[l][u] < thr2;
                other = other || (nr && jg0 + u != ig[l]);
                r2[l][u] = nr ? __builtin_inff() : r2[l][u];
            }
        near |= __builtin_amdgcn_ballot_w64(other);
    }
#pragma unroll
    for (int l = 0; l < ILP; ++l) {
        constexpr int KB = ACC > 0 ? ACC : G;
#pragma unroll
        for (int u0 = 0; u0 < G; u0 += KB) {
            float y0 = ACC ? -L[l].c0 : L[l].s0;
            float y1 = ACC ? -L[l].c1 : L[l].s1;
            float y2 = ACC ? -L[l].c2 : L[l].s2;
#pragma unroll
            for (int u = u0; u < u0 + KB; ++u) {
                const float rinv = __builtin_amdgcn_rsqf(r2[l][u]);
                const float rinv2 = rinv * rinv;
                const float rinv3 = rinv2 * rinv;
                float A, Bt;
                if (TENSOR == T_OSEEN) {
                    A = rinv;
                    Bt = rinv3;
                } else {
                    A = fmaf(gamma, rinv3, rinv);
                    Bt = rinv3 * fmaf(m3g, rinv2, kc.one);
                }
                const float dF = fmaf(dx[l][u], fjx[u], fmaf(dy[l][u], fjy[u], dz[l][u] * fjz[u]));
                const float sB = Bt * dF;
                y0 = fmaf(A, fjx[u], fmaf(sB, dx[l][u], y0));
                y1 = fmaf(A, fjy[u], fmaf(sB, dy[l][u], y1));
                y2 = fmaf(A, fjz[u], fmaf(sB, dz[l][u], y2));
            }
            if (ACC) {
                const float t0 = L[l].s0 + y0;
                const float t1 = L[l].s1 + y1;
                const float t2 = L[l].s2 + y2;
                L[l].c0 = (t0 - L[l].s0) - y0;
                L[l].c1 = (t1 - L[l].s1) - y1;
                L[l].c2 = (t2 - L[l].s2) - y2;
                L[l].s0 = t0;
                L[l].s1 = t1;
                L[l].s2 = t2;
            } else {
                L[l].s0 = y0;
                L[l].s1 = y1;
                L[l].s2 = y2;
            }
        }
    }
}

// j-side partials of one tile: the ROWS = BLOCK / 16 row sums of each element
// and component added in FP64, in row order, stored as FP32 at jpart[c][I][p].
template <int BLOCK>
__device__ __forceinline__ void sym_tile_rows(const float* s_jacc, float* __restrict__ jpart,
                                              const SymShape& sh, int ib, int pt)
{
    constexpr int ROWS = BLOCK / 16;
    for (int t = (int)threadIdx.x; t < 3 * SYM_TJ; t += BLOCK) {
        const int k = t / SYM_TJ, e = t % SYM_TJ;
        double sum = 0.0;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) sum += (double)s_jacc[(k * ROWS + r) * SYM_TJ + e];
        jpart[((size_t)k * sh.nb + ib) * (size_t)sh.lmax + (size_t)(pt + e)] = (float)sum;
    }
}

// Minimum resident waves per SIMD the register allocation must allow: four
// with work-groups of 256 or 512 lanes (40 / 64 KiB of LDS: four / two
// work-groups per CU); 128-lane groups (28 KiB) reach at most three.
template <int BLOCK>
struct SymWaves {
    static constexpr int value = BLOCK >= 256 ? 4 : 2;
};

// Near flags.  Row W = ib * RB + w (RB = B / SYM_RUN rows per i-block, w the
// wave) holds one 16-byte entry per tile t of the block's virtual j range:
// the lanes of wave w that met a near pair with that tile (64 bits: a lane
// holds particles tid and tid + BLOCK) and the chunks of 16 j particles of the
// tile they were met in (8 bits).  After the rows, one 16-byte entry per W:
// the lanes that met a near pair within their own block (the diagonal
// work-group) and the chunks of 16 particles of the block (32 bits).  Every call writes every entry it covers (zero if nothing was
// met), so nothing is cleared and no earlier call's entries are ever read.
template <int BLOCK, int ILP>
__device__ __forceinline__ uint4* sym_flag_row(uint8_t* __restrict__ flags, const SymShape& sh,
                                               int ib)
{
    constexpr int RB = BLOCK * ILP / SYM_RUN;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    return (uint4*)flags + (size_t)(ib * RB + w) * (size_t)sh.nt;
}

__device__ __forceinline__ void sym_flag_tile(uint4* __restrict__ frow, int t, uint64_t lanes,
                                              uint32_t chunks)
{
    if ((threadIdx.x & 63) == 0) {
        uint32_t* e = (uint32_t*)(frow + t);
        *(uint2*)e = make_uint2((uint32_t)lanes, (uint32_t)(lanes >> 32));
        e[2] = chunks;
    }
}

template <int BLOCK, int ILP>
__device__ __forceinline__ void sym_flag_diag(uint8_t* __restrict__ flags, const SymShape& sh,
                                              int ib, uint64_t lanes, uint32_t chunks)
{
    constexpr int RB = BLOCK * ILP / SYM_RUN;
    const size_t rows = (size_t)sh.nb * RB;
    uint4* d = (uint4*)flags + rows * (size_t)sh.nt;
    if ((threadIdx.x & 63) == 0)
        d[ib * RB + (int)(threadIdx.x >> 6)] =
            make_uint4((uint32_t)lanes, (uint32_t)(lanes >> 32), chunks, 0u);
}

// ILP particles per lane (ILP 2: the i-block of BLOCK * ILP particles has
// particle tid and tid + BLOCK in lane tid), groups of U steps.
// flags: near flags per wave and tile (see sym_flag_row).
template <int TENSOR, int ACC, int BLOCK, int ILP, bool PER>
__global__ void __launch_bounds__(BLOCK, SymWaves<BLOCK>::value)
k_pair_f32_sym(const float4* __restrict__ pos, const float4* __restrict__ frc, int n, SymShape sh,
               PairConst pc, double* __restrict__ partial, float* __restrict__ jpart,
               uint8_t* __restrict__ flags)
{
    constexpr int B = BLOCK * ILP;   // particles per block
    constexpr int U = ILP == 1 ? 8 : 4;
    static_assert(B % SYM_TJ == 0, "j tiles must not straddle blocks");
    constexpr int ROWS = BLOCK / 16;
    constexpr int TS = 2 * SYM_TJ;                      // slots of one staged tile
    constexpr int NSLOT = 2 * TS > B ? 2 * TS : B;      // two tiles, or one diagonal block
    constexpr int LOADS = (2 * SYM_TJ + BLOCK - 1) / BLOCK;   // tile records per thread
    __shared__ float4 s_pos[NSLOT];
    __shared__ float4 s_frc[NSLOT];
    __shared__ float s_jacc[3 * ROWS * SYM_TJ];
    const int tid = threadIdx.x;
    // work-groups: the nb diagonal blocks first, then split-major (see sym_shape)
    const bool diag = (int)blockIdx.x < sh.nb;
    int ib, s;
    if (diag) {
        ib = (int)blockIdx.x;
        s = sh.isplits;
    } else {
        const int w = (int)blockIdx.x - sh.nb;
        s = w / sh.nb;
        ib = w - s * sh.nb;
    }
    SymLane L[ILP];
    sym_lanes_init<ILP, BLOCK, PER>(L, pos, n, ib);
    const VConst kc = vconst(pc);
    const float4 far_j4 = make_float4(far_j<PER>(), far_j<PER>(), far_j<PER>(), 0.0f);
    const float4 zero4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint64_t near = 0;

    if (diag) {
        // the i-block with itself: every ordered pair, one-sided, in groups of
        // four (compensation at least every four terms)
        constexpr int ACC_D = ACC > 4 ? 4 : ACC;
        constexpr int G = 4;
        uint32_t dch = 0;   // chunks of 16 j of the block with a near pair
        const int jt = ib * B;
        int ig[ILP];
#pragma unroll
        for (int r = 0; r < ILP; ++r) {
            const int t = tid + r * BLOCK;
            ig[r] = jt + t;
            float4 rp = far_j4, rf = zero4;
            if (jt + t < n) {
                rp = pos[jt + t];
                rf = frc[jt + t];
            }
            s_pos[t] = rp;
            s_frc[t] = rf;
        }
        __syncthreads();
#pragma unroll 1
        for (int k = 0; k < B; k += G) {
            float4 pj[G], fj[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                pj[u] = s_pos[k + u];
                fj[u] = s_frc[k + u];
            }
            uint64_t nd = 0;
            diag_group<TENSOR, ACC_D, G, ILP, PER>(L, ig, pj, fj, jt + k, kc, nd);
            if (nd != 0) {
                near |= nd;
                dch |= 1u << (k / 16);
            }
        }
        sym_flag_diag<BLOCK, ILP>(flags, sh, ib, near, dch);
        sym_lanes_store<ILP, BLOCK>(L, n, ib, s, pc.alpha_sum, partial);
        return;
    }

    float fi[ILP][3];
#pragma unroll
    for (int l = 0; l < ILP; ++l) {
        const int i = ib * B + tid + l * BLOCK;
        fi[l][0] = fi[l][1] = fi[l][2] = 0.0f;
        if (i < n) {
            const float4 f = frc[i];
            fi[l][0] = f.x;
            fi[l][1] = f.y;
            fi[l][2] = f.z;
        }
    }
    float y[ILP][3];
    const int q = tid & 15;
    const int row = tid >> 4;
    const int half = sh.nb >> 1;
    const int lI = (sh.h + ((sh.extra && ib < half) ? 1 : 0)) * B;
    const int pbeg = sh.off[s] * SYM_TJ;
    const int pend = min(lI, sh.off[s + 1] * SYM_TJ);
    uint4* const frow = sym_flag_row<BLOCK, ILP>(flags, sh, ib);
    // block J and first particle of the tile at virtual position pt
    auto tile_block = [&](int pt) { return (ib + 1 + pt / B) % sh.nb; };
    // this thread's records of the tile at pt: element e of record r is
    // position (r < SYM_TJ) or force of particle jt + (r mod SYM_TJ)
    auto tile_load = [&](int pt, float4 (&rec)[LOADS]) {
        const int jt = tile_block(pt) * B + (pt % B);
#pragma unroll
        for (int m = 0; m < LOADS; ++m) {
            const int r = tid + m * BLOCK;
            const int j = jt + (r & (SYM_TJ - 1));
            const float4* src = r < SYM_TJ ? pos : frc;
            const float fill = r < SYM_TJ ? far_j<PER>() : 0.0f;
            rec[m] = make_float4(fill, fill, fill, 0.0f);
            if (r < 2 * SYM_TJ && j < n) rec[m] = src[j];
        }
    };
    // chunk c of a tile at slots c * 32 + e and c * 32 + 16 + e
    auto tile_store = [&](int buf, const float4 (&rec)[LOADS]) {
#pragma unroll
        for (int m = 0; m < LOADS; ++m) {
            const int r = tid + m * BLOCK;
            if (r < 2 * SYM_TJ) {
                const int e = r & (SYM_TJ - 1);
                float4* dst = (r < SYM_TJ ? s_pos : s_frc) + buf * TS + (e >> 4) * 32 + (e & 15);
                dst[0] = rec[m];
                dst[16] = rec[m];
            }
        }
    };
    float4 rec[LOADS];
    if (pbeg < pend) {
        tile_load(pbeg, rec);
        tile_store(0, rec);
    }
    // the lane's own records are waited for here, once: a wait inside the
    // chunk loop would also wait for the next tile's loads in flight
#pragma unroll
    for (int l = 0; l < ILP; ++l)
        asm volatile("" : "+v"(L[l].x), "+v"(L[l].y), "+v"(L[l].z), "+v"(fi[l][0]), "+v"(fi[l][1]),
                     "+v"(fi[l][2]));
    __syncthreads();
#pragma unroll 1
    for (int pt = pbeg, buf = 0; pt < pend; pt += SYM_TJ, buf ^= 1) {
        const bool more = pt + SYM_TJ < pend;
        if (more) tile_load(pt + SYM_TJ, rec);   // consumed after the chunk loop
        uint32_t nch = 0;   // chunks of the tile with a near pair
#pragma unroll 1
        for (int c = 0; c < SYM_TJ / 16; ++c) {
            float aj0, aj1, aj2;
            const float4* sp = s_pos + buf * TS + c * 32 + q;
            const float4* sf = s_frc + buf * TS + c * 32 + q;
            uint64_t nc = 0;
            StaticFor<0, 16 / U>::run([&](auto g_c) {
                constexpr int K0 = decltype(g_c)::value * U;
                sym_steps<TENSOR, ACC, PER, K0, U, ILP>(L, fi, y, aj0, aj1, aj2, sp, sf, kc, nc);
            });
            if (nc != 0) {
                near |= nc;
                nch |= 1u << c;
            }
            s_jacc[(0 * ROWS + row) * SYM_TJ + c * 16 + q] = aj0;
            s_jacc[(1 * ROWS + row) * SYM_TJ + c * 16 + q] = aj1;
            s_jacc[(2 * ROWS + row) * SYM_TJ + c * 16 + q] = aj2;
        }
        if (more) tile_store(buf ^ 1, rec);
        sym_flag_tile(frow, pt / SYM_TJ, near, nch);
        near = 0;
        __syncthreads();   // the tile's j-side sums are complete, the next tile is staged
        sym_tile_rows<BLOCK>(s_jacc, jpart, sh, ib, pt);
        __syncthreads();   // s_jacc is free for the next tile
    }
    sym_lanes_store<ILP, BLOCK>(L, n, ib, s, pc.alpha_sum, partial);
}

// Variant 2 with its chunk in assembly (sym_chunk_asm.h, generated by
// gen_sym_chunk.py): 256 lanes, two particles per lane, Kahan blocks of 16
// terms (one per chunk).  Same block schedule, near-pair flags, j-side rows
// and outputs as k_pair_f32_sym; the tiles are staged as six doubled float
// arrays (x, y, z of positions and forces), so that every component is read
// into a register of the parity the generated code expects.
template <int TENSOR, int ACC, bool PER>
__global__ void __launch_bounds__(256, 4)
k_pair_f32_sym_asm(const float4* __restrict__ pos, const float4* __restrict__ frc, int n,
                   SymShape sh, PairConst pc, double* __restrict__ partial,
                   float* __restrict__ jpart, uint8_t* __restrict__ flags)
{
    constexpr int BLOCK = 256, ILP = 2, B = 512, ROWS = BLOCK / 16;
    constexpr int TS = 2 * SYM_TJ;     // floats of one doubled array of a tile
    // two tiles of six doubled arrays (2 x 6 x 256), or one block of six
    // plain arrays (6 x 512) for the diagonal work-groups
    __shared__ float s_soa[2 * 6 * TS];
    __shared__ float s_jacc[3 * ROWS * SYM_TJ];
    typedef __attribute__((address_space(3))) float lds_float;
    const int tid = threadIdx.x;
    const bool diag = (int)blockIdx.x < sh.nb;
    int ib, s;
    if (diag) {
        ib = (int)blockIdx.x;
        s = sh.isplits;
    } else {
        const int w = (int)blockIdx.x - sh.nb;
        s = w / sh.nb;
        ib = w - s * sh.nb;
    }
    SymLane L[ILP];
    sym_lanes_init<ILP, BLOCK, PER>(L, pos, n, ib);
    const VConst kc = vconst(pc);
    uint64_t near = 0;

    if (diag) {
        constexpr int G = 4;
        uint32_t dch = 0;   // chunks of 16 j of the block with a near pair
        const int jt = ib * B;
        int ig[ILP];
#pragma unroll
        for (int r = 0; r < ILP; ++r) {
            const int t = tid + r * BLOCK;
            ig[r] = jt + t;
            float4 rp = make_float4(far_j<PER>(), far_j<PER>(), far_j<PER>(), 0.0f);
            float4 rf = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (jt + t < n) {
                rp = pos[jt + t];
                rf = frc[jt + t];
            }
            s_soa[0 * B + t] = rp.x;
            s_soa[1 * B + t] = rp.y;
            s_soa[2 * B + t] = rp.z;
            s_soa[3 * B + t] = rf.x;
            s_soa[4 * B + t] = rf.y;
            s_soa[5 * B + t] = rf.z;
        }
        __syncthreads();
#pragma unroll 1
        for (int k = 0; k < B; k += G) {
            float4 pj[G], fj[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                pj[u] = make_float4(s_soa[0 * B + k + u], s_soa[1 * B + k + u],
                                    s_soa[2 * B + k + u], 0.0f);
                fj[u] = make_float4(s_soa[3 * B + k + u], s_soa[4 * B + k + u],
                                    s_soa[5 * B + k + u], 0.0f);
            }
            uint64_t nd = 0;
            diag_group<TENSOR, 4, G, ILP, PER>(L, ig, pj, fj, jt + k, kc, nd);
            if (nd != 0) {
                near |= nd;
                dch |= 1u << (k / 16);
            }
        }
        sym_flag_diag<BLOCK, ILP>(flags, sh, ib, near, dch);
        sym_lanes_store<ILP, BLOCK>(L, n, ib, s, pc.alpha_sum, partial);
        return;
    }

    // lane state in the registers the generated chunk expects
    float x0 = L[0].x, y0 = L[0].y, z0 = L[0].z, x1 = L[1].x, y1 = L[1].y, z1 = L[1].z;
    float f0x = 0.0f, f0y = 0.0f, f0z = 0.0f, f1x = 0.0f, f1y = 0.0f, f1z = 0.0f;
    {
        const int i0 = ib * B + tid, i1 = i0 + BLOCK;
        if (i0 < n) {
            const float4 f = frc[i0];
            f0x = f.x;
            f0y = f.y;
            f0z = f.z;
        }
        if (i1 < n) {
            const float4 f = frc[i1];
            f1x = f.x;
            f1y = f.y;
            f1z = f.z;
        }
    }
    float s0x = 0.0f, s0y = 0.0f, s0z = 0.0f, s1x = 0.0f, s1y = 0.0f, s1z = 0.0f;   // sums
    float n0x = 0.0f, n0y = 0.0f, n0z = 0.0f, n1x = 0.0f, n1y = 0.0f, n1z = 0.0f;   // -compensation
    float k_gamma = kc.gamma, k_m3g = kc.m3g, k_thr2 = kc.thr2, k_inf = __builtin_inff();
    asm volatile("" : "+v"(k_inf));
    uint64_t nearl = 0;   // lanes that met a near pair in the tile
    uint32_t nearf = 0;   // chunks of the tile they were met in
    const int q = tid & 15;
    const int row = tid >> 4;
    const int half = sh.nb >> 1;
    const int lI = (sh.h + ((sh.extra && ib < half) ? 1 : 0)) * B;
    const int pbeg = sh.off[s] * SYM_TJ;
    const int pend = min(lI, sh.off[s + 1] * SYM_TJ);
    uint4* const frow = sym_flag_row<BLOCK, ILP>(flags, sh, ib);
    auto tile_block = [&](int pt) { return (ib + 1 + pt / B) % sh.nb; };
    // this thread's record of the tile at pt: position (tid < SYM_TJ) or force
    // of particle jt + tid mod SYM_TJ
    auto tile_load = [&](int pt) {
        const int jt = tile_block(pt) * B + (pt % B);
        const int j = jt + (tid & (SYM_TJ - 1));
        const float4* src = tid < SYM_TJ ? pos : frc;
        const float fill = tid < SYM_TJ ? far_j<PER>() : 0.0f;
        float4 r = make_float4(fill, fill, fill, 0.0f);
        if (j < n) r = src[j];
        return r;
    };
    // element e of chunk c at slots c * 32 + e and c * 32 + 16 + e of its array
    auto tile_store = [&](int buf, float4 r) {
        const int e = tid & (SYM_TJ - 1);
        float* dst = s_soa + (buf * 6 + (tid < SYM_TJ ? 0 : 3)) * TS + (e >> 4) * 32 + (e & 15);
        dst[0] = r.x;
        dst[16] = r.x;
        dst[TS] = r.y;
        dst[TS + 16] = r.y;
        dst[2 * TS] = r.z;
        dst[2 * TS + 16] = r.z;
    };
    // the next tile is read from HBM a whole tile ahead: its load is issued
    // right after the previous one was staged, before the j-side row stores
    float4 rec = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (pbeg < pend) tile_store(0, tile_load(pbeg));
    if (pbeg + SYM_TJ < pend) rec = tile_load(pbeg + SYM_TJ);
    __syncthreads();
#pragma unroll 1
    for (int pt = pbeg, buf = 0; pt < pend; pt += SYM_TJ, buf ^= 1) {
        const bool more = pt + SYM_TJ < pend;
        // the tile's 8 chunks in one statement: every operand is in/out, so the
        // values stay in the registers the generated code names, with no copies;
        // the j-side sums of each chunk go to this row's slots of s_jacc
        uint32_t addr = (uint32_t)(uintptr_t)(lds_float*)(s_soa + buf * 6 * TS + q);
        uint32_t jaddr = (uint32_t)(uintptr_t)(lds_float*)(s_jacc + row * SYM_TJ + q);
        uint32_t cnt, stmp;
        const uint32_t kmask = ACC == 32 ? 1u : 0u;   // Kahan after every chunk or every second
#define SD_SYM_TILE_CALL(TEXT)                                                                 \
    asm volatile(TEXT                                                                          \
                 : [s0x] "+" SD_SYM_R_S0x(s0x), [s0y] "+" SD_SYM_R_S0y(s0y),                   \
                   [s0z] "+" SD_SYM_R_S0z(s0z), [s1x] "+" SD_SYM_R_S1x(s1x),                   \
                   [s1y] "+" SD_SYM_R_S1y(s1y), [s1z] "+" SD_SYM_R_S1z(s1z),                   \
                   [y0x] "+" SD_SYM_R_Y0x(n0x), [y0y] "+" SD_SYM_R_Y0y(n0y),                   \
                   [y0z] "+" SD_SYM_R_Y0z(n0z), [y1x] "+" SD_SYM_R_Y1x(n1x),                   \
                   [y1y] "+" SD_SYM_R_Y1y(n1y), [y1z] "+" SD_SYM_R_Y1z(n1z),                   \
                   [x0] "+" SD_SYM_R_X0x(x0), [y0] "+" SD_SYM_R_X0y(y0), [z0] "+" SD_SYM_R_X0z(z0), \
                   [x1] "+" SD_SYM_R_X1x(x1), [y1] "+" SD_SYM_R_X1y(y1), [z1] "+" SD_SYM_R_X1z(z1), \
                   [f0x] "+" SD_SYM_R_FI0x(f0x), [f0y] "+" SD_SYM_R_FI0y(f0y),                 \
                   [f0z] "+" SD_SYM_R_FI0z(f0z), [f1x] "+" SD_SYM_R_FI1x(f1x),                 \
                   [f1y] "+" SD_SYM_R_FI1y(f1y), [f1z] "+" SD_SYM_R_FI1z(f1z),                 \
                   [adr] "+" SD_SYM_R_ADDR(addr), [jadr] "+" SD_SYM_R_JADDR(jaddr),            \
                   [nf] "+s"(nearf), [nl] "+s"(nearl), [cnt] "=&s"(cnt), [tmp] "=&s"(stmp)     \
                 : [gam] SD_SYM_R_GAMMA(k_gamma), [thr] SD_SYM_R_THR2(k_thr2),                 \
                   [thro] SD_SYM_R_THR2O(k_thr2), [inf] SD_SYM_R_INF(k_inf),                   \
                   [m3g] SD_SYM_R_M3G(k_m3g), [kmask] "s"(kmask)                               \
                 : SD_SYM_CLOBBERS, "vcc", "scc", "memory")
        if constexpr (TENSOR == T_RPY && !PER)
            SD_SYM_TILE_CALL(SD_SYM_TILE_RPY_FREE);
        else if constexpr (TENSOR == T_RPY)
            SD_SYM_TILE_CALL(SD_SYM_TILE_RPY_PER);
        else if constexpr (!PER)
            SD_SYM_TILE_CALL(SD_SYM_TILE_OSEEN_FREE);
        else
            SD_SYM_TILE_CALL(SD_SYM_TILE_OSEEN_PER);
#undef SD_SYM_TILE_CALL
        if (more) {
            tile_store(buf ^ 1, rec);
            if (pt + 2 * SYM_TJ < pend) rec = tile_load(pt + 2 * SYM_TJ);
        }
        sym_flag_tile(frow, pt / SYM_TJ, nearl, nearf);
        nearl = 0;
        nearf = 0;
        __syncthreads();   // the tile's j-side sums are complete, the next tile is staged
        sym_tile_rows<BLOCK>(s_jacc, jpart, sh, ib, pt);
        __syncthreads();   // s_jacc is free for the next tile
    }
    // i side: S - C = S + NC (the negated compensation)
    L[0].s0 = s0x;
    L[0].s1 = s0y;
    L[0].s2 = s0z;
    L[1].s0 = s1x;
    L[1].s1 = s1y;
    L[1].s2 = s1z;
    L[0].c0 = -n0x;
    L[0].c1 = -n0y;
    L[0].c2 = -n0z;
    L[1].c0 = -n1x;
    L[1].c1 = -n1y;
    L[1].c2 = -n1z;
    sym_lanes_store<ILP, BLOCK>(L, n, ib, s, pc.alpha_sum, partial);
}

// FP64 difference x_i - x_j of a near pair (i: position xi of the FP32
// record): from the FP64 positions when given (nearest image in a box), else
// from the FP32 records (exact difference of floats, or the fixed-point
// difference times s).
template <bool PER>
__device__ __forceinline__ void near_diff_v(float xi, float yi, float zi, int i, float4 pj, int jg,
                                            const PairConst& pc, const double* __restrict__ x64,
                                            double& d0, double& d1, double& d2)
{
    if (x64) {
        d0 = x64[3 * (size_t)i + 0] - x64[3 * (size_t)jg + 0];
        d1 = x64[3 * (size_t)i + 1] - x64[3 * (size_t)jg + 1];
        d2 = x64[3 * (size_t)i + 2] - x64[3 * (size_t)jg + 2];
        if (PER) nearest_image_d(pc, d0, d1, d2);
    } else if (PER) {
        d0 = (double)(int)(__float_as_uint(xi) - __float_as_uint(pj.x)) * pc.s_q;
        d1 = (double)(int)(__float_as_uint(yi) - __float_as_uint(pj.y)) * pc.s_q;
        d2 = (double)(int)(__float_as_uint(zi) - __float_as_uint(pj.z)) * pc.s_q;
    } else {
        d0 = (double)xi - (double)pj.x;
        d1 = (double)yi - (double)pj.y;
        d2 = (double)zi - (double)pj.z;
    }
}

// Last split row of variant 2, one wave per run S of SYM_RUN particles
// (lane: particle q = S SYM_RUN + lane, at offset o of its block J):
//  * the j side: the FP32 partials of the blocks I that took block J,
//    added in FP64 in a fixed order (I = J - 1, J - 2, ..., then the
//    antipode), times alpha_sum;
//  * the near pairs: every candidate the near flags name (see below) below
//    the FP32 near threshold (the test of the pair kernel, so exactly the
//    masked pairs), j != q, evaluated in FP64 (near_term) in the order of
//    the candidate list.
template <int TENSOR, bool PER>
__global__ void __launch_bounds__(SYM_RUN)
k_sym_fold_near(const float* __restrict__ jpart, const float4* __restrict__ pos,
                const float4* __restrict__ frc, const double* __restrict__ x64, int n, int B,
                int wpb, SymShape sh, PairConst pc, const uint8_t* __restrict__ flags,
                double* __restrict__ out, const double* __restrict__ partial, double mu0,
                double* __restrict__ vel)
{
    constexpr int FOLD_CAP = 256;   // candidates listed before their records are loaded
    __shared__ float4 s_pos[FOLD_CAP];
    __shared__ float4 s_frc[FOLD_CAP];
    __shared__ double s_x64[3 * FOLD_CAP];   // FP64 positions when x64 is given
    __shared__ int s_idx[FOLD_CAP];
    // one wave per run S of SYM_RUN particles; particle q at offset o of block J
    const int S = blockIdx.x, lane = threadIdx.x;
    const int q = S * SYM_RUN + lane;
    const int J = (S * SYM_RUN) / B;
    const int o = q - J * B;
    const int nb = sh.nb, half = nb >> 1;
    const size_t cs = (size_t)nb * (size_t)sh.lmax;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    if (q < n) {
        // blocks I = J - d (d = 1 .. h) in that order, the loads of a group of
        // them issued before its adds
        constexpr int G = 8;
        for (int d0 = 1; d0 <= sh.h; d0 += G) {
            float a[G][3];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int d = d0 + u;
                if (d <= sh.h) {
                    const int I = (J - d + nb) % nb;
                    const size_t at = (size_t)I * sh.lmax + (size_t)(d - 1) * B + o;
                    a[u][0] = jpart[at];
                    a[u][1] = jpart[cs + at];
                    a[u][2] = jpart[2 * cs + at];
                }
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (d0 + u <= sh.h) {
                    v0 += (double)a[u][0];
                    v1 += (double)a[u][1];
                    v2 += (double)a[u][2];
                }
            }
        }
        if (sh.extra) {
            const int I = (J + half) % nb;
            if (I < half) {
                const size_t at = (size_t)I * sh.lmax + (size_t)sh.h * B + o;
                v0 += (double)jpart[at];
                v1 += (double)jpart[cs + at];
                v2 += (double)jpart[2 * cs + at];
            }
        }
    }
    v0 *= pc.alpha_sum;
    v1 *= pc.alpha_sum;
    v2 *= pc.alpha_sum;
    // near pairs of q.  The flags name candidate particles; they are listed in
    // LDS in a fixed order (the diagonal block, the flagged chunks of the tiles
    // in the row of q's wave: q's block as i-block, then the flagged lanes of
    // the waves of preceding blocks whose entry for q's tile names a chunk of
    // q's run: q's block as j-block), their records are loaded together once
    // FOLD_CAP are listed or the list ends, and every q tests every listed
    // candidate (the FP32 threshold test again, then FP64).  A pair of
    // different blocks lies in the virtual range of exactly one of the two,
    // and each source lists a particle once, so every near pair is found once.
    const float thr2 = pc.thr2_f;
    float xq = far_i<PER>(), yq = far_i<PER>(), zq = far_i<PER>();
    double xq64[3] = { 0.0, 0.0, 0.0 };
    if (q < n) {
        const float4 p = pos[q];
        xq = p.x;
        yq = p.y;
        zq = p.z;
        if (x64) {
            xq64[0] = x64[3 * (size_t)q];
            xq64[1] = x64[3 * (size_t)q + 1];
            xq64[2] = x64[3 * (size_t)q + 2];
        }
    }
    int cnt = 0;   // listed candidates (the same in every lane)
    uint32_t psub = 0, pco = 0;   // this lane's pairs against the premise r >= 2a
    auto flush = [&]() {
        __syncthreads();
        for (int k = lane; k < cnt; k += SYM_RUN) {
            const int jg = s_idx[k];
            const bool in = jg < n;
            s_pos[k] = in ? pos[jg] : make_float4(far_j<PER>(), far_j<PER>(), far_j<PER>(), 0.0f);
            s_frc[k] = in ? frc[jg] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (x64) {
                s_x64[3 * k] = in ? x64[3 * (size_t)jg] : 0.0;
                s_x64[3 * k + 1] = in ? x64[3 * (size_t)jg + 1] : 0.0;
                s_x64[3 * k + 2] = in ? x64[3 * (size_t)jg + 2] : 0.0;
            }
        }
        __syncthreads();
        // the FP32 test for groups of 8 candidates, then the pairs it found
        // in ascending order
        for (int e0 = 0; e0 < cnt; e0 += 8) {
            uint32_t nm = 0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (e0 + u < cnt) {
                    const float4 pj = s_pos[e0 + u];
                    const float dx = pdiff<PER>(xq, pj.x);
                    const float dy = pdiff<PER>(yq, pj.y);
                    const float dz = pdiff<PER>(zq, pj.z);
                    if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < thr2) nm |= 1u << u;
                }
            }
            for (; nm != 0u; nm &= nm - 1u) {
                const int e = e0 + __builtin_ctz(nm);
                const float4 pj = s_pos[e];
                const int jg = s_idx[e];
                if (jg != q && q < n && jg < n) {
                    const float4 fj = s_frc[e];
                    double d0, d1, d2;
                    if (x64) {   // the FP64 positions, staged
                        d0 = xq64[0] - s_x64[3 * e];
                        d1 = xq64[1] - s_x64[3 * e + 1];
                        d2 = xq64[2] - s_x64[3 * e + 2];
                        if (PER) nearest_image_d(pc, d0, d1, d2);
                    } else {
                        near_diff_v<PER>(xq, yq, zq, q, pj, jg, pc, nullptr, d0, d1, d2);
                    }
                    const int cls = near_term<TENSOR>(pc, d0, d1, d2, (double)fj.x, (double)fj.y,
                                                      (double)fj.z, v0, v1, v2);
                    if (q < jg) {
                        psub += cls == PREMISE_SUB2A;
                        pco += cls == PREMISE_COINCIDENT;
                    }
                }
            }
        }
        __syncthreads();
        cnt = 0;
    };
    auto add_range = [&](int j0, int len) {   // particles j0 .. j0 + len - 1, len <= 64
        if (cnt + len > FOLD_CAP) flush();
        if (lane < len) s_idx[cnt + lane] = j0 + lane;
        cnt += len;
    };
    const int RB = B / SYM_RUN;          // runs (= flag rows) per block
    const int r = S - J * RB;            // q's run within its block
    const int w = r % wpb;               // the wave that holds it
    const int ilp = RB / wpb;
    const int nt = sh.nt;
    const size_t rows = (size_t)nb * RB;
    const int TB = B / SYM_TJ;           // tiles per block
    const uint4* ftile = (const uint4*)flags;
    const uint4* fdiag = ftile + rows * (size_t)nt;
    for (uint32_t ch = fdiag[J * RB + w].z; ch != 0u; ch &= ch - 1u)
        add_range(J * B + 16 * __builtin_ctz(ch), 16);
    const int ntJ = (sh.h + ((sh.extra && J < half) ? 1 : 0)) * TB;
    const uint4* frow = ftile + (size_t)(J * RB + w) * nt;
    // (the entries are read by all lanes at once and handed out with readlane:
    // a load per flagged entry would put a memory latency in the chain)
    for (int t0 = 0; t0 < ntJ; t0 += 64) {
        const uint32_t chl = t0 + lane < ntJ ? frow[t0 + lane].z : 0u;
        uint64_t m = __builtin_amdgcn_ballot_w64(chl != 0u);
        while (m) {
            const int k = __builtin_ctzll(m);
            m &= m - 1;
            const int pt = (t0 + k) * SYM_TJ;
            const int jt = ((J + 1 + pt / B) % nb) * B + pt % B;
            for (uint32_t ch = __builtin_amdgcn_readlane(chl, k); ch != 0u; ch &= ch - 1u)
                add_range(jt + 16 * __builtin_ctz(ch), 16);
        }
    }
    // q's block J is block d of the virtual range of I = J - d (d = 1 .. h),
    // and block h + 1 of I = J + nb / 2 when nb is even and I < nb / 2; q's
    // run covers chunks c0 .. c0 + 3 of its tile tq
    const int tq = (r * SYM_RUN) / SYM_TJ;
    const uint32_t rch = 0xFu << (((r * SYM_RUN) % SYM_TJ) / 16);
    const int Ie = (J + half) % nb;
    const int dmax = sh.h + ((sh.extra && Ie < half) ? 1 : 0);
    for (int c0 = 0; c0 < dmax * wpb; c0 += 64) {
        uint4 ev = make_uint4(0u, 0u, 0u, 0u);
        const int c = c0 + lane;          // c = (d - 1) wpb + w'
        if (c < dmax * wpb) {
            const int d = c / wpb + 1, wp = c % wpb;
            const int I = (J - d + nb) % nb;
            ev = ftile[(size_t)(I * RB + wp) * nt + (size_t)((d - 1) * TB + tq)];
        }
        uint64_t m = __builtin_amdgcn_ballot_w64((ev.z & rch) != 0u);
        while (m) {
            const int k = __builtin_ctzll(m);
            m &= m - 1;
            const int cc = c0 + k;
            const int d = cc / wpb + 1, wp = cc % wpb;
            const int I = (J - d + nb) % nb;
            const uint64_t lanes = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(ev.y, k) << 32) |
                                   (uint32_t)__builtin_amdgcn_readlane(ev.x, k);
            // lane k of wave w' holds particles I B + l BLOCK + 64 w' + k
            const int add = __builtin_popcountll(lanes) * ilp;
            if (cnt + add > FOLD_CAP) flush();
            const int at = __builtin_popcountll(lanes & ((1ull << lane) - 1ull));
            if ((lanes >> lane) & 1)
                for (int l = 0; l < ilp; ++l)
                    s_idx[cnt + at * ilp + l] = I * B + l * (wpb * SYM_RUN) + wp * SYM_RUN + lane;
            cnt += add;
        }
    }
    if (cnt > 0) flush();
    count_premise_lanes(psub, pco);
    if (q < n) {
        if (vel) {
            // the merge: mu0 F + rows 0 .. isplits in order + this row (k_merge's sum)
            const float4 fq = frc[q];
            double w0 = mu0 * (double)fq.x, w1 = mu0 * (double)fq.y, w2 = mu0 * (double)fq.z;
            add_split_rows(partial, sh.isplits + 1, n, q, w0, w1, w2);
            vel[3 * (size_t)q + 0] = w0 + v0;
            vel[3 * (size_t)q + 1] = w1 + v1;
            vel[3 * (size_t)q + 2] = w2 + v2;
        } else {
            out[q] = v0;
            out[(size_t)n + q] = v1;
            out[2 * (size_t)n + q] = v2;
        }
    }
}

// ---------------------------------------------------------------- FP64 path

template <int TENSOR, int BLOCK, bool PER>
__global__ void __launch_bounds__(BLOCK)
k_pair_f64_lds(const double4* __restrict__ pos, const double4* __restrict__ frc, int n, int jchunk,
               int S, PairConst pc, double* __restrict__ partial)
{
    __shared__ double4 s_pos[BLOCK];
    __shared__ double4 s_frc[BLOCK];
    int ib, s;
    map_block(S, ib, s);
    const int tid = threadIdx.x;
    const int i = ib * BLOCK + tid;
    double xi0 = -1.0e15, xi1 = -1.0e15, xi2 = -1.0e15;
    if (i < n) {
        const double4 p = pos[i];
        xi0 = p.x;
        xi1 = p.y;
        xi2 = p.z;
    }
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;  // scaled far-field sums
    double n0 = 0.0, n1 = 0.0, n2 = 0.0;  // near sums (physical units)
    const int jbeg = s * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const double gamma = pc.gamma, m3g = -3.0 * pc.gamma, thr2 = pc.thr2_d;
    const double4 far_j = make_double4(1.0e15, 1.0e15, 1.0e15, 0.0);
    const double4 zero4 = make_double4(0.0, 0.0, 0.0, 0.0);
    double4 rp = far_j, rf = zero4;
    if (jbeg + tid < jend) {
        rp = pos[jbeg + tid];
        rf = frc[jbeg + tid];
    }
    for (int jt = jbeg; jt < jend; jt += BLOCK) {
        __syncthreads();
        s_pos[tid] = rp;
        s_frc[tid] = rf;
        __syncthreads();
        const int jn = jt + BLOCK + tid;
        rp = far_j;
        rf = zero4;
        if (jn < jend) {
            rp = pos[jn];
            rf = frc[jn];
        }
        for (int k = 0; k < BLOCK; ++k) {
            const double4 pj = s_pos[k];
            const double4 fj = s_frc[k];
            double dx = xi0 - pj.x, dy = xi1 - pj.y, dz = xi2 - pj.z;
            if (PER) {  // nearest image; an exact half-box difference may take either image
                dx = fma(-pc.box, rint(dx * pc.ibox), dx);
                dy = fma(-pc.box, rint(dy * pc.ibox), dy);
                dz = fma(-pc.box, rint(dz * pc.ibox), dz);
            }
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const bool nr = r2 < thr2;
            double rinv = rsqrt(r2);
            rinv = nr ? 0.0 : rinv;
            const double rinv2 = rinv * rinv;
            const double rinv3 = rinv2 * rinv;
            double A, Bt;
            if (TENSOR == T_OSEEN) {
                A = rinv;
                Bt = rinv3;
            } else {
                A = fma(gamma, rinv3, rinv);
                Bt = rinv3 * fma(m3g, rinv2, 1.0);
            }
            const double sB = Bt * fma(dx, fj.x, fma(dy, fj.y, dz * fj.z));
            v0 = fma(A, fj.x, fma(sB, dx, v0));
            v1 = fma(A, fj.y, fma(sB, dy, v1));
            v2 = fma(A, fj.z, fma(sB, dz, v2));
            if (nr && (jt + k) != i && i < n && (jt + k) < n) {
                const int cls = near_term<TENSOR>(pc, dx, dy, dz, fj.x, fj.y, fj.z, n0, n1, n2);
                count_premise(i < jt + k ? cls : PREMISE_OK);
            }
        }
    }
    if (i < n) {
        const size_t base = (size_t)s * 3 * (size_t)n + (size_t)i;
        partial[base] = pc.alpha * v0 + n0;
        partial[base + (size_t)n] = pc.alpha * v1 + n1;
        partial[base + 2 * (size_t)n] = pc.alpha * v2 + n2;
    }
}

// ------------------------------------------------------------------ merge

template <typename F4>
__global__ void __launch_bounds__(256)
k_merge(const double* __restrict__ partial, int S, int n, const F4* __restrict__ frc, double mu0,
        double* __restrict__ vel)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const F4 f = frc[i];
    double v0 = mu0 * (double)f.x, v1 = mu0 * (double)f.y, v2 = mu0 * (double)f.z;
    add_split_rows(partial, S, n, i, v0, v1, v2);
    vel[3 * (size_t)i + 0] = v0;
    vel[3 * (size_t)i + 1] = v1;
    vel[3 * (size_t)i + 2] = v2;
}

// ---------------------------------------------------------------- launchers

template <int TENSOR, int ACC, int BLOCK, int ILP>
static hipError_t launch_f32_t(const PairLaunch& L, const float4* pos, const float4* frc,
                               const double* x64, int n, const PairConst& pc, double* partial,
                               hipStream_t st)
{
    const int iblocks = (n + BLOCK * ILP - 1) / (BLOCK * ILP);
    dim3 grid(iblocks * L.splits), block(BLOCK);
    if (pc.box > 0.0) {
        if (L.variant == 1)
            hipLaunchKernelGGL((k_pair_f32_smem<TENSOR, ACC, BLOCK, ILP, true>), grid, block, 0,
                               st, pos, frc, x64, n, L.jchunk, L.splits, pc, partial);
        else
            hipLaunchKernelGGL((k_pair_f32_lds<TENSOR, ACC, BLOCK, ILP, true>), grid, block, 0,
                               st, pos, frc, x64, n, L.jchunk, L.splits, pc, partial);
    } else {
        if (L.variant == 1)
            hipLaunchKernelGGL((k_pair_f32_smem<TENSOR, ACC, BLOCK, ILP, false>), grid, block, 0,
                               st, pos, frc, x64, n, L.jchunk, L.splits, pc, partial);
        else
            hipLaunchKernelGGL((k_pair_f32_lds<TENSOR, ACC, BLOCK, ILP, false>), grid, block, 0,
                               st, pos, frc, x64, n, L.jchunk, L.splits, pc, partial);
    }
    return hipGetLastError();
}

template <int TENSOR, int ACC, int BLOCK, int ILP>
static hipError_t launch_f32_sym(const PairLaunch& L, const float4* pos, const float4* frc, int n,
                                 const PairConst& pc, double* partial, hipStream_t st)
{
    const SymShape sh = sym_shape_of(L, n);
    float* jpart = (float*)((char*)partial + sym_jpart_offset(L, n));
    uint8_t* flags = (uint8_t*)partial + sym_flags_offset(L, n);
    dim3 grid(sh.nb * sh.isplits + sh.nb), block(BLOCK);
    if constexpr (ACC == 16 || ACC == 32) {
        static_assert(BLOCK == 256 && ILP == 2, "Kahan blocks of 16 or 32: the assembly shape");
        // the shape with its chunk in assembly
        if (pc.box > 0.0)
            hipLaunchKernelGGL((k_pair_f32_sym_asm<TENSOR, ACC, true>), grid, block, 0, st, pos,
                               frc, n, sh, pc, partial, jpart, flags);
        else
            hipLaunchKernelGGL((k_pair_f32_sym_asm<TENSOR, ACC, false>), grid, block, 0, st, pos,
                               frc, n, sh, pc, partial, jpart, flags);
    } else {
        if (pc.box > 0.0)
            hipLaunchKernelGGL((k_pair_f32_sym<TENSOR, ACC, BLOCK, ILP, true>), grid, block, 0,
                               st, pos, frc, n, sh, pc, partial, jpart, flags);
        else
            hipLaunchKernelGGL((k_pair_f32_sym<TENSOR, ACC, BLOCK, ILP, false>), grid, block, 0,
                               st, pos, frc, n, sh, pc, partial, jpart, flags);
    }
    return hipGetLastError();
}

hipError_t launch_pair_fold(const PairLaunch& L, int tensor, const float4* pos, const float4* frc,
                            const double* x64, int n, const PairConst& pc, double* partial,
                            hipStream_t st, double mu0, double* vel)
{
    if (L.variant != 2) return hipSuccess;
    const SymShape sh = sym_shape_of(L, n);
    const float* jpart = (const float*)((const char*)partial + sym_jpart_offset(L, n));
    uint8_t* flags = (uint8_t*)partial + sym_flags_offset(L, n);
    double* out = partial + (size_t)(sh.isplits + 1) * 3 * (size_t)n;
    const int B = L.block * L.ilp;
    const bool per = pc.box > 0.0;
#define SD_FOLD(T, P)                                                                      \
    hipLaunchKernelGGL((k_sym_fold_near<T, P>), dim3(sh.nb * (B / SYM_RUN)), dim3(SYM_RUN), 0, \
                       st, jpart, pos, frc, x64, n, B, L.block / 64, sh, pc, flags, out,   \
                       partial, mu0, vel)
    if (tensor == T_OSEEN) {
        if (per) SD_FOLD(T_OSEEN, true); else SD_FOLD(T_OSEEN, false);
    } else {
        if (per) SD_FOLD(T_RPY, true); else SD_FOLD(T_RPY, false);
    }
#undef SD_FOLD
    return hipGetLastError();
}

template <int TENSOR, int ACC>
static hipError_t launch_f32_b(const PairLaunch& L, const float4* pos, const float4* frc,
                               const double* x64, int n, const PairConst& pc, double* partial,
                               hipStream_t st)
{
    if (L.variant == 2) {
        if constexpr (ACC == 16 || ACC == 32) {   // the assembly shape only
            if (L.block == 256 && L.ilp == 2)
                return launch_f32_sym<TENSOR, ACC, 256, 2>(L, pos, frc, n, pc, partial, st);
        } else if constexpr (ACC == 0 || ACC == 4 || ACC == 8) {
            if (L.block == 128 && L.ilp == 1)
                return launch_f32_sym<TENSOR, ACC, 128, 1>(L, pos, frc, n, pc, partial, st);
            if (L.block == 256 && L.ilp == 1)
                return launch_f32_sym<TENSOR, ACC, 256, 1>(L, pos, frc, n, pc, partial, st);
            if (L.block == 512 && L.ilp == 1)
                return launch_f32_sym<TENSOR, ACC, 512, 1>(L, pos, frc, n, pc, partial, st);
            if (L.block == 128 && L.ilp == 2)
                return launch_f32_sym<TENSOR, ACC, 128, 2>(L, pos, frc, n, pc, partial, st);
            if (L.block == 256 && L.ilp == 2)
                return launch_f32_sym<TENSOR, ACC, 256, 2>(L, pos, frc, n, pc, partial, st);
        }
        return hipErrorInvalidValue;
    }
    if constexpr (ACC <= 8) {   // Kahan blocks of 16: variant 2 only
#define SD_CASE(B, I)                                                                        \
    if (L.block == B && L.ilp == I)                                                          \
        return launch_f32_t<TENSOR, ACC, B, I>(L, pos, frc, x64, n, pc, partial, st);
        SD_CASE(64, 1) SD_CASE(128, 1) SD_CASE(256, 1)
        SD_CASE(64, 2) SD_CASE(128, 2) SD_CASE(256, 2)
#undef SD_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pair_f32(const PairLaunch& L, int tensor, int acc, const float4* pos,
                           const float4* frc, const double* x64, int n, const PairConst& pc,
                           double* partial, hipStream_t st)
{
#define SD_ACC(T)                                                                    \
    switch (acc) {                                                                   \
    case 0: return launch_f32_b<T, 0>(L, pos, frc, x64, n, pc, partial, st);         \
    case 1: return launch_f32_b<T, 1>(L, pos, frc, x64, n, pc, partial, st);         \
    case 2: return launch_f32_b<T, 2>(L, pos, frc, x64, n, pc, partial, st);         \
    case 4: return launch_f32_b<T, 4>(L, pos, frc, x64, n, pc, partial, st);         \
    case 8: return launch_f32_b<T, 8>(L, pos, frc, x64, n, pc, partial, st);         \
    case 16: return launch_f32_b<T, 16>(L, pos, frc, x64, n, pc, partial, st);       \
    case 32: return launch_f32_b<T, 32>(L, pos, frc, x64, n, pc, partial, st);       \
    default: return hipErrorInvalidValue;                                            \
    }
    if (tensor == T_OSEEN) { SD_ACC(T_OSEEN) }
    SD_ACC(T_RPY)
#undef SD_ACC
}

template <int TENSOR, int BLOCK>
static hipError_t launch_f64_t(const PairLaunch& L, const double4* pos, const double4* frc, int n,
                               const PairConst& pc, double* partial, hipStream_t st)
{
    dim3 grid(((n + BLOCK - 1) / BLOCK) * L.splits), block(BLOCK);
    if (pc.box > 0.0)
        hipLaunchKernelGGL((k_pair_f64_lds<TENSOR, BLOCK, true>), grid, block, 0, st, pos, frc, n,
                           L.jchunk, L.splits, pc, partial);
    else
        hipLaunchKernelGGL((k_pair_f64_lds<TENSOR, BLOCK, false>), grid, block, 0, st, pos, frc,
                           n, L.jchunk, L.splits, pc, partial);
    return hipGetLastError();
}

hipError_t launch_pair_f64(const PairLaunch& L, int tensor, const double4* pos, const double4* frc,
                           int n, const PairConst& pc, double* partial, hipStream_t st)
{
#define SD_CASE(B)                                                                           \
    if (L.block == B)                                                                        \
        return tensor == T_OSEEN ? launch_f64_t<T_OSEEN, B>(L, pos, frc, n, pc, partial, st) \
                                 : launch_f64_t<T_RPY, B>(L, pos, frc, n, pc, partial, st);
    SD_CASE(64) SD_CASE(128) SD_CASE(256) SD_CASE(512)
#undef SD_CASE
    return hipErrorInvalidValue;
}

__global__ void k_premise_clear(unsigned long long* c)
{
    if (threadIdx.x < 2) c[threadIdx.x] = 0ull;
}

hipError_t premise_counts(int64_t* sub2a, int64_t* coincident, bool reset, hipStream_t st)
{
    // the counters of the current device (each device holds its own copy)
    void* dev = nullptr;
    hipError_t e = hipGetSymbolAddress(&dev, HIP_SYMBOL(g_premise));
    if (e != hipSuccess) return e;
    unsigned long long h[2] = { 0ull, 0ull };
    if ((e = hipMemcpyAsync(h, dev, sizeof h, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if (reset) {
        hipLaunchKernelGGL(k_premise_clear, dim3(1), dim3(64), 0, st, (unsigned long long*)dev);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (sub2a) *sub2a = (int64_t)h[0];
    if (coincident) *coincident = (int64_t)h[1];
    return hipSuccess;
}

hipError_t launch_merge_f32(const double* partial, int splits, int n, const float4* frc, double mu0,
                            double* vel, hipStream_t st)
{
    hipLaunchKernelGGL((k_merge<float4>), dim3((n + 255) / 256), dim3(256), 0, st, partial, splits,
                       n, frc, mu0, vel);
    return hipGetLastError();
}

hipError_t launch_merge_f64(const double* partial, int splits, int n, const double4* frc,
                            double mu0, double* vel, hipStream_t st)
{
    hipLaunchKernelGGL((k_merge<double4>), dim3((n + 255) / 256), dim3(256), 0, st, partial,
                       splits, n, frc, mu0, vel);
    return hipGetLastError();
}

}  // namespace sd
