// autotune.cpp -- sd_autotune: time candidate shapes of the pair kernel on a
// synthetic configuration of n particles and install the fastest.
//
// Inputs: a simple cubic lattice at volume fraction 0.05 (spacing 4.37a, so
// the timed loop is the far-field fast path, as in a dilute suspension) with a
// fixed pattern of unit forces.  Candidates: kernel variant (LDS tiles /
// scalar cache / pair symmetry), work-group size, particles per lane, Kahan
// block (FP32_KAHAN) and the number of j-range splits, plus the automatic
// choice itself, so the installed entry is never one that timed slower than
// it.  Each candidate is warmed up once and timed over three launches with
// HIP events on the caller's stream.
#include "sd.h"
#include "sd_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace sd;

namespace {

struct Cand {
    sd_kernel_config c;
    float ms;
};

bool same_config(const sd_kernel_config& a, const sd_kernel_config& b)
{
    return a.variant == b.variant && a.block == b.block && a.splits == b.splits &&
           a.ilp == b.ilp && a.kahan_block == b.kahan_block;
}

std::vector<sd_kernel_config> candidates(int32_t prec, int64_t n)
{
    std::vector<sd_kernel_config> out;
    const sd_kernel_config d = default_config(prec, n);
    std::vector<int> split_opts;
    for (int s : { d.splits / 2, d.splits, d.splits * 2, d.splits * 4 })
        if (s >= 1) split_opts.push_back(s);
    std::sort(split_opts.begin(), split_opts.end());
    split_opts.erase(std::unique(split_opts.begin(), split_opts.end()), split_opts.end());
    const int variants = prec == SD_FP64 ? 1 : 2;
    for (int v = 0; v < variants; ++v)
        for (int block : { 64, 128, 256 })
            for (int ilp : { 1, 2 }) {
                if (prec == SD_FP64 && ilp != 1) continue;
                std::vector<int> kbs;
                if (prec == SD_FP32_KAHAN) kbs = { 1, 2, 4, 8 };
                else kbs = { 0 };
                for (int kb : kbs)
                    for (int s : split_opts) {
                        if (kb == 8 && block < 128) continue;
                        // keep the same number of j-tiles per split across block sizes
                        int splits = std::max(1, (int)((int64_t)s * 256 / block));
                        const int64_t tiles = (n + block - 1) / block;
                        splits = (int)std::min<int64_t>(splits, tiles);
                        sd_kernel_config c;
                        c.variant = v;
                        c.block = block;
                        c.ilp = ilp;
                        c.kahan_block = kb;
                        c.splits = splits;
                        out.push_back(c);
                    }
            }
    // variant 2 (pair symmetry), FP32 only, when its j-side workspace fits:
    // 128-512 lanes with one or two particles per lane, Kahan blocks of 4 or
    // 8 (the compiled chunk loop) and, with 256 lanes and two particles per
    // lane, 16 or 32 (the chunk loop in assembly); requested split counts of
    // 8 to 64
    if (prec != SD_FP64)
        for (int block : { 128, 256, 512 })
            for (int ilp : { 1, 2 }) {
                if (block * ilp > 512 || !sym_fits(n, block * ilp)) continue;
                sd_kernel_config c;
                c.variant = 2;
                c.block = block;
                c.ilp = ilp;
                std::vector<int> kbs = { 0 };
                if (prec == SD_FP32_KAHAN) {
                    kbs = { 4, 8 };
                    if (block == 256 && ilp == 2) kbs.insert(kbs.end(), { 16, 32 });
                }
                for (int kb : kbs)
                    for (int s : { 8, 16, 32, 64 }) {
                        c.kahan_block = kb;
                        c.splits = s;
                        out.push_back(c);
                    }
            }
    // the automatic choice, timed last (after the clocks have ramped up)
    out.erase(std::remove_if(out.begin(), out.end(),
                             [&](const sd_kernel_config& c) { return same_config(c, d); }),
              out.end());
    out.push_back(d);
    return out;
}

}  // namespace

extern "C" sd_status sd_autotune(const sd_params* p, int64_t n, int32_t precision, void* stream,
                                 char* report, int64_t report_len)
{
    sd_status st;
    if ((st = check_params(p)) || (st = check_n(n)) || (st = check_precision(precision))) return st;
    hipStream_t hs = (hipStream_t)stream;
    const bool f64 = precision == SD_FP64;
    const size_t rec = f64 ? 32 : 16;
    // synthetic inputs
    const double spacing = std::cbrt(4.0 * M_PI / 3.0 / 0.05) * p->a;
    const int64_t side = (int64_t)std::ceil(std::cbrt((double)n));
    std::vector<double> h((size_t)n * 8, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t ix = i % side, iy = (i / side) % side, iz = i / (side * side);
        h[8 * i + 0] = (ix - 0.5 * side) * spacing;
        h[8 * i + 1] = (iy - 0.5 * side) * spacing;
        h[8 * i + 2] = (iz - 0.5 * side) * spacing;
        h[8 * i + 4] = std::sin(0.7 * (double)i);
        h[8 * i + 5] = std::cos(1.3 * (double)i);
        h[8 * i + 6] = -1.0;
    }
    std::vector<unsigned char> up((size_t)n * 2 * rec);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 4; ++k) {
            if (f64) {
                ((double*)up.data())[4 * i + k] = h[8 * i + k];
                ((double*)up.data())[4 * (n + i) + k] = h[8 * i + 4 + k];
            } else {
                ((float*)up.data())[4 * i + k] = (float)h[8 * i + k];
                ((float*)up.data())[4 * (n + i) + k] = (float)h[8 * i + 4 + k];
            }
        }
    void* buf = nullptr;
    if ((st = ws_get(WS_TUNE, up.size() + 3 * (size_t)n * sizeof(double), &buf))) return st;
    void* pos = buf;
    void* frc = (char*)buf + (size_t)n * rec;
    double* vel = (double*)((char*)buf + up.size());
    if (hipMemcpyAsync(buf, up.data(), up.size(), hipMemcpyHostToDevice, hs) != hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess)
        return fail(SD_EDEVICE, "autotune upload failed");

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(SD_EDEVICE, "hipEventCreate failed");
    // each candidate is timed with the configuration forced; the automatic
    // choice is restored afterwards
    std::vector<Cand> res;
    for (const sd_kernel_config& c : candidates(precision, n)) {
        if (check_config(precision, c) != SD_OK) continue;
        if ((st = sd_set_kernel_config(precision, &c))) break;
        if ((st = mobility_apply(p, n, pos, frc, vel, precision, stream))) break;
        (void)hipEventRecord(e0, hs);
        for (int r = 0; r < 3; ++r)
            if ((st = mobility_apply(p, n, pos, frc, vel, precision, stream))) break;
        (void)hipEventRecord(e1, hs);
        if (st) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
            st = fail(SD_EDEVICE, "autotune timing failed");
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        res.push_back({ c, ms / 3.0f });
    }
    sd_set_kernel_config(precision, nullptr);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    if (res.empty()) return fail(SD_EUNSUPPORTED, "no candidate configuration ran");
    std::sort(res.begin(), res.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
    set_tuned_config(precision, n, res[0].c);
    const sd_kernel_config d = default_config(precision, n);
    double default_ms = -1.0;   // -1: the automatic choice did not run
    for (const Cand& r : res)
        if (same_config(r.c, d)) default_ms = r.ms;
    if (report && report_len > 0) {
        char dl[64];
        snprintf(dl, sizeof dl, "%.4f", default_ms);
        std::string s = "{\"n\": " + std::to_string(n) + ", \"precision\": " +
                        std::to_string(precision) + ", \"candidates\": " +
                        std::to_string(res.size()) + ", \"default_ms\": " + dl +
                        ", \"ranked\": [";
        for (size_t k = 0; k < res.size() && k < 12; ++k) {
            char line[256];
            snprintf(line, sizeof line,
                     "%s{\"variant\": %d, \"block\": %d, \"splits\": %d, \"ilp\": %d, "
                     "\"kahan_block\": %d, \"ms\": %.4f}",
                     k ? ", " : "", res[k].c.variant, res[k].c.block, res[k].c.splits,
                     res[k].c.ilp, res[k].c.kahan_block, res[k].ms);
            s += line;
        }
        s += "]}";
        const size_t m = std::min<size_t>(s.size(), (size_t)report_len - 1);
        memcpy(report, s.data(), m);
        report[m] = 0;
    }
    return SD_OK;
}
