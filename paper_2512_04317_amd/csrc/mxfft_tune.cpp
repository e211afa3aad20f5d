// mxfft_tune.cpp -- launch autotuner of the generic line kernels (lines per
// work-group, and for n <= 64 the single-launch kernel against them) and its
// plain-text cache (one JSON object per line, keyed by GPU architecture, n,
// format and block size).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "mxfft.h"
#include "mxfft_internal.hpp"

namespace {

struct Entry {
    std::string arch;
    int n = 0, format = 0, block = 0, lines = 0, single = 0, stats = 0, chunks = 0;
    double ms = 0.0;
};

// every MX element format (MXFP8 and MXFP6) keys its cache entries by block size
bool is_mx(int format)
{
    return format == MXFFT_E4M3 || format == MXFFT_E5M2 || format == MXFFT_E2M3 || format == MXFFT_E3M2;
}

// Value of "key": in one line; false when absent or malformed.
bool find_num(const std::string& line, const char* key, double* v)
{
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = line.find(k);
    if (at == std::string::npos) return false;
    const char* p = line.c_str() + at + k.size();
    char* end = nullptr;
    *v = std::strtod(p, &end);
    return end != p;
}

bool find_str(const std::string& line, const char* key, std::string* v)
{
    const std::string k = std::string("\"") + key + "\":";
    size_t at = line.find(k);
    if (at == std::string::npos) return false;
    at = line.find('"', at + k.size());
    if (at == std::string::npos) return false;
    const size_t e = line.find('"', at + 1);
    if (e == std::string::npos) return false;
    *v = line.substr(at + 1, e - at - 1);
    return true;
}

bool parse(const std::string& line, Entry* e)
{
    double n, f, b, l, ms;
    if (!find_str(line, "arch", &e->arch)) return false;
    if (!find_num(line, "n", &n) || !find_num(line, "format", &f) || !find_num(line, "block", &b) ||
        !find_num(line, "lines", &l) || !find_num(line, "ms", &ms))
        return false;
    e->n = (int)n;
    e->format = (int)f;
    e->block = (int)b;
    e->lines = (int)l;
    e->ms = ms;
    double one = 0.0;   // keys absent in older entries: the defaults
    e->single = find_num(line, "single", &one) ? (int)one : 0;
    e->stats = find_num(line, "stats", &one) ? (int)one : 0;
    e->chunks = find_num(line, "chunks", &one) ? (int)one : 0;
    return true;
}

std::string format_entry(const Entry& e)
{
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "{\"arch\": \"%s\", \"n\": %d, \"format\": %d, \"block\": %d, \"lines\": %d, \"ms\": %.6f, "
                  "\"single\": %d, \"stats\": %d, \"chunks\": %d}",
                  e.arch.c_str(), e.n, e.format, e.block, e.lines, e.ms, e.single, e.stats, e.chunks);
    return buf;
}

std::vector<std::string> read_lines(const char* path)
{
    std::vector<std::string> out;
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line))
        if (!line.empty()) out.push_back(line);
    return out;
}

bool same_key(const Entry& a, const Entry& b)
{
    return a.arch == b.arch && a.n == b.n && a.format == b.format && a.block == b.block;
}

Entry key_of(const char* arch, int n, const mxfft_params* p)
{
    Entry k;
    k.arch = arch;
    k.n = n;
    k.format = p->format;
    k.block = is_mx(p->format) ? p->block : 0;
    return k;
}

// Rewrite the cache with `e` replacing any entry of the same key.
bool store(const char* path, const Entry& e)
{
    std::vector<std::string> lines = read_lines(path);
    std::ostringstream os;
    for (const std::string& l : lines) {
        Entry o;
        if (parse(l, &o) && same_key(o, e)) continue;
        os << l << "\n";
    }
    os << format_entry(e) << "\n";
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return false;
        f << os.str();
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

std::string arch_name()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    return prop.gcnArchName;
}

}  // namespace

extern "C" {

mxfft_status mxfft_tune_cache_lookup(const char* cache_path, const char* arch, int32_t n, const mxfft_params* p,
                                     mxfft_tuning* out)
{
    if (!cache_path || !arch || !p || !out) return MXFFT_EINVAL;
    const Entry key = key_of(arch, n, p);
    for (const std::string& l : read_lines(cache_path)) {
        Entry e;
        if (parse(l, &e) && same_key(e, key)) {
            out->lines = e.lines;
            out->fast = 0;
            out->ms = e.ms;
            out->single = (n <= mxk::kSmallN) ? e.single : 0;
            out->stats = e.stats;
            out->chunks = e.chunks;
            return MXFFT_OK;
        }
    }
    return MXFFT_EINVAL;
}

mxfft_status mxfft_tune(int32_t n, const mxfft_params* p, int32_t sample, const char* cache_path,
                        uint32_t tune_flags, mxfft_tuning* out, void* stream)
{
    if (!p || !out || sample < 1) return MXFFT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    mxfft_plan_t plan = nullptr;
    mxfft_status st = mxfft_plan(&plan, n, sample, p, stream);
    if (st != MXFFT_OK) return st;
    mxfft_tuning cur{};
    mxfft_plan_get_tuning(plan, &cur);
    const std::string arch = arch_name();
    if (cache_path && !(tune_flags & MXFFT_TUNE_FORCE)) {
        mxfft_tuning hit{};
        if (mxfft_tune_cache_lookup(cache_path, arch.c_str(), n, p, &hit) == MXFFT_OK &&
            mxfft_plan_set_tuning(plan, &hit) == MXFFT_OK) {
            *out = hit;
            out->fast = cur.fast;
            return mxfft_plan_destroy(plan);
        }
    }

    const size_t count = (size_t)sample * n * n;
    float2 *x = nullptr, *y = nullptr;
    int32_t* k = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = hipMalloc((void**)&x, count * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc((void**)&y, count * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc((void**)&k, (size_t)sample * sizeof(int32_t)) == hipSuccess;
    ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    ok = ok && mxk::launch_fill(x, count, 0x5EEDu + (uint32_t)n, s) == hipSuccess;

    // candidates.  Line kernels: the default lines and its halvings down to
    // 1, and for n <= 64 the single-launch kernel.  Register-resident passes:
    // where the row pass can gather Alg. 1's statistics, that against the
    // separate statistics read; the read with work-groups per slice by batch
    // (0) or fixed at 1, 4, 16 (while a chunk keeps >= 1024 values and the
    // sample's statistics fit the workspace)
    std::vector<mxfft_tuning> cand;
    if (cur.fast) {
        const bool pre = !(p->flags & MXFFT_NO_PRESCALE);
        mxfft_tuning t{};
        if (cur.stats == 0) cand.push_back(t);   // fused statistics
        t.stats = 1;
        if (pre) {
            for (int c : {0, 1, 4, 16}) {
                if (c && ((long)n * n / c < 1024 || (size_t)c * sample > mxk::stats_parts(n, sample))) continue;
                t.chunks = c;
                cand.push_back(t);
            }
        }
        if (cand.empty()) cand.push_back(mxfft_tuning{});
        if (n <= mxk::kSmallN) {   // 128^2: the single launch against the register-resident passes
            mxfft_tuning one{};
            one.single = 1;
            cand.push_back(one);
        }
    } else {
        for (int r = mxk::line_lines_per_group(n); r >= 1 && (int)cand.size() < 5; r /= 2) {
            mxfft_tuning t{};
            t.lines = r;
            cand.push_back(t);
        }
        if (n <= mxk::kSmallN) {
            mxfft_tuning t{};
            t.single = 1;
            cand.push_back(t);
        }
    }
    // timing: the GPU first runs the default for at least 20 ms (clocks up
    // from idle), then the candidates take turns, one call each per round,
    // so that clock drift touches them all alike; median over 5 rounds
    auto timed_call = [&](float* t_ms) {
        bool r = hipEventRecord(e0, s) == hipSuccess;
        r = r && mxfft_forward(plan, x, y, sample, k, stream) == MXFFT_OK;
        r = r && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        return r && hipEventElapsedTime(t_ms, e0, e1) == hipSuccess;
    };
    std::vector<char> usable(cand.size(), 0);
    for (size_t c = 0; c < cand.size() && ok; c++) {
        usable[c] = mxfft_plan_set_tuning(plan, &cand[c]) == MXFFT_OK;
        float t_ms = 0.f;
        if (usable[c]) ok = timed_call(&t_ms);   // first call of each candidate: warm-up
    }
    if (ok) {
        const mxfft_tuning d{};
        ok = mxfft_plan_set_tuning(plan, &cand[0]) == MXFFT_OK || mxfft_plan_set_tuning(plan, &d) == MXFFT_OK;
        float spent = 0.f;
        for (int w = 0; w < 200 && ok && spent < 20.f; w++) {
            float t_ms = 0.f;
            ok = timed_call(&t_ms);
            spent += t_ms;
        }
    }
    std::vector<std::vector<float>> ms(cand.size());
    for (int round = 0; round < 5 && ok; round++)
        for (size_t c = 0; c < cand.size() && ok; c++) {
            if (!usable[c]) continue;
            float t_ms = 0.f;
            ok = mxfft_plan_set_tuning(plan, &cand[c]) == MXFFT_OK && timed_call(&t_ms);
            ms[c].push_back(t_ms);
        }
    mxfft_tuning best = cand[0], best_lines = cand[0];
    double best_ms = 1e30, best_lines_ms = 1e30;
    for (size_t c = 0; c < cand.size() && ok; c++) {
        if (ms[c].empty()) continue;
        std::sort(ms[c].begin(), ms[c].end());
        const double med = ms[c][ms[c].size() / 2];
        const mxfft_tuning& t = cand[c];
        if (med < best_ms) {
            best_ms = med;
            best = t;
        }
        if (!cur.fast && !t.single && med < best_lines_ms) {
            best_lines_ms = med;
            best_lines = t;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(x);
    (void)hipFree(y);
    (void)hipFree(k);
    mxfft_plan_destroy(plan);
    if (!ok) return MXFFT_EHIP;
    *out = best;
    out->fast = cur.fast;
    out->ms = best_ms;
    if (!cur.fast) out->lines = best_lines.lines;   // the line-kernel choice, even when single wins
    if (cache_path) {
        Entry e = key_of(arch.c_str(), n, p);
        e.lines = out->lines;
        e.single = out->single;
        e.stats = out->stats;
        e.chunks = out->chunks;
        e.ms = best_ms;
        if (!store(cache_path, e)) return MXFFT_EINVAL;
    }
    return MXFFT_OK;
}

}  // extern "C"
